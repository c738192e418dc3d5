// Canonical order of the point ids inside every bin of a deterministic plan.
//
// The plan-time scatter places each merged point's id in its bin through an
// atomic cursor, so the order of the ids inside a bin depends on the timing of
// the scatter.  A deterministic plan sorts the ids of every bin by value once
// after the scatter: the bin runs (fixed-length slices of each bin's list) and
// the order in which a run's points are spread are then functions of the plan
// descriptor alone, and two plans of one descriptor evaluate bit for bit alike.
// The ids are sorted in slices of whole bins (at most kSliceKeys ids, or one
// larger bin) by rocPRIM's segmented radix sort, one segment per bin.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "pgc_internal.h"

namespace pgc {

namespace {
constexpr int64_t kSliceKeys = int64_t(1) << 27;  // 1 GiB of ids per sorting slice
}

// `begin` holds nbins + 1 offsets (bin b is [begin[b], begin[b + 1]) of ids);
// the ids use bits [0, end_bit).  Temporaries are freed before returning.
hipError_t sort_bin_ids(unsigned long long* ids, const std::vector<unsigned long long>& begin, int end_bit,
                        hipStream_t s)
{
    const int64_t nbins = (int64_t)begin.size() - 1;
    if (nbins <= 0) return hipSuccess;
    // slices of whole bins
    std::vector<int64_t> cut{0};
    for (int64_t b = 0; b < nbins; ++b) {
        const unsigned long long lo = begin[cut.back()], hi = begin[b + 1];
        if (b > cut.back() && hi - lo > (unsigned long long)kSliceKeys) cut.push_back(b);
    }
    cut.push_back(nbins);
    int64_t max_keys = 0, max_segs = 0;
    for (size_t k = 0; k + 1 < cut.size(); ++k) {
        max_keys = std::max<int64_t>(max_keys, (int64_t)(begin[cut[k + 1]] - begin[cut[k]]));
        max_segs = std::max<int64_t>(max_segs, cut[k + 1] - cut[k]);
    }
    if (max_keys > 0xffffffffll || max_segs > 0x7fffffffll) return hipErrorInvalidValue;
    if (max_keys == 0) return hipSuccess;

    unsigned long long* out = nullptr;
    unsigned int* offs = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipMalloc(&out, (size_t)max_keys * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&offs, (size_t)(max_segs + 1) * sizeof(unsigned int));
    std::vector<unsigned int> h((size_t)max_segs + 1);
    for (size_t k = 0; k + 1 < cut.size() && e == hipSuccess; ++k) {
        const int64_t b0 = cut[k], b1 = cut[k + 1];
        const unsigned long long base = begin[b0];
        const unsigned int keys = (unsigned int)(begin[b1] - base);
        const unsigned int segs = (unsigned int)(b1 - b0);
        if (keys == 0) continue;
        for (int64_t b = b0; b <= b1; ++b) h[b - b0] = (unsigned int)(begin[b] - base);
        size_t need = 0;
        e = rocprim::segmented_radix_sort_keys(nullptr, need, ids + base, out, keys, segs, offs, offs + 1, 0,
                                               (unsigned int)end_bit, s);
        if (e != hipSuccess) break;
        if (need > tmp_bytes) {
            if (tmp) (void)hipFree(tmp);
            tmp = nullptr;
            tmp_bytes = 0;
            if ((e = hipMalloc(&tmp, need)) != hipSuccess) break;
            tmp_bytes = need;
        }
        // the host offsets are reused by the next slice: wait for this one
        e = hipMemcpyAsync(offs, h.data(), (size_t)(segs + 1) * sizeof(unsigned int), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = rocprim::segmented_radix_sort_keys(tmp, need, ids + base, out, keys, segs, offs, offs + 1, 0,
                                                   (unsigned int)end_bit, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ids + base, out, (size_t)keys * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                               s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (tmp) (void)hipFree(tmp);
    if (offs) (void)hipFree(offs);
    if (out) (void)hipFree(out);
    return e;
}

}  // namespace pgc
