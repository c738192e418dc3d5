// pgc_coeffs_to_q_static: the evaluation of pgc_coeffs_to_q with every
// per-call buffer (nodal values, loss field, fine grid, transform buffers,
// partial sums) taken from one static device array instead of the plan's
// workspace, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "pgc.h"
#include "pgc_internal.h"

// Each device that loads the library holds its own copy of this array until
// the process ends.  In host code `scratch` names a host-side stand-in, never
// a device address: kernels receive the address hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[PGC_STATIC_SCRATCH_BYTES];

namespace pgc {
namespace {

constexpr size_t kScratchAlign = 256;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// Lay the evaluation's buffers out from `base` (nullptr: only count bytes) and
// return the bytes used.  The buffers are those of the plan's Workspace that
// one evaluation touches, with the same sizes.
size_t carve(const Plan& p, char* base, Workspace* ws)
{
    size_t off = 0;
    auto take = [&](int64_t bytes) -> void* {
        void* ptr = base ? static_cast<void*>(base + off) : nullptr;
        off += ((size_t)bytes + kScratchAlign - 1) / kScratchAlign * kScratchAlign;
        return ptr;
    };
    const bool fp64 = p.precision == PGC_PRECISION_FP64;
    int64_t nsym = 1;
    for (int l = 0; l < p.dim; ++l) nsym *= p.np;
    Workspace w;
    w.cin = static_cast<double*>(take(p.Nd * 8));
    w.P = static_cast<double*>(take(p.nid * 8));
    w.G = static_cast<double*>(take(p.nid * 8));
    w.Gg = fp64 ? static_cast<void*>(w.G) : take(p.nid * (int64_t)p.elt);
    w.H = static_cast<double*>(take(p.nid * 8));
    w.tmpA = static_cast<double*>(take(p.tmp_elems * 8));
    w.tmpB = static_cast<double*>(take(p.tmp_elems * 8));
    w.qminus = static_cast<double*>(take(p.Nd * 8));
    w.qplus = static_cast<double*>(take(p.Nd * 8));
    w.red = static_cast<double*>(take(64 * 8));
    if (p.gain_mode == kGainSlab) {
        w.sym = take(nsym * (int64_t)p.elt);
        w.partial = take((int64_t)p.n_chunks * p.ngd * 8);
        w.grid = static_cast<double*>(take(p.ngd * 8));
    } else {
        w.grid64 = static_cast<double*>(take(p.ngd * 8));
    }
    if (ws) *ws = w;
    return off;
}

}  // namespace
}  // namespace pgc

extern "C" pgc_status pgc_coeffs_to_q_static(pgc_plan plan, const void* coeffs, void* q, void* qplus,
                                             void* stream)
{
    if (!plan || !coeffs || !q) return PGC_ERR_INVALID_ARG;
    const pgc::Plan& p = plan->p;
    if (pgc::carve(p, nullptr, nullptr) > (size_t)PGC_STATIC_SCRATCH_BYTES) return PGC_ERR_SCRATCH;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pgc::status_of(e);
    if (dev != p.device) return PGC_ERR_INVALID_ARG;
    void* base = nullptr;
    e = pgc::scratch_address(dev, &base);
    if (e != hipSuccess) return pgc::status_of(e);
    pgc::Workspace ws;
    pgc::carve(p, static_cast<char*>(base), &ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = pgc::launch_synthesis(p, ws, coeffs, s);
    if (e == hipSuccess) e = pgc::launch_loss(p, ws, s);
    if (e == hipSuccess) e = pgc::launch_gain(p, ws, q, qplus, s);
    return pgc::status_of(e);
}
