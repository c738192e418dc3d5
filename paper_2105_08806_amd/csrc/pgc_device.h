// Device-side pieces shared by the gain kernels of single plans and of
// batches: fine-grid folding, the per-point geometry of a merged collision
// point, its kernel values, its orbit sum and its bin.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pgc_internal.h"

namespace pgc {
namespace {

__device__ __forceinline__ int fold_index(int t, int nh)
{
    // reflection of an unfolded grid index into [0, nh]: the images -z and
    // 2 pi - z of a point z in [0, pi] land on -t and 2 nh - t.
    return t < 0 ? -t : (t > nh ? 2 * nh - t : t);
}

template <typename T>
struct GainParams {
    const T* v1;        // n_i interior node velocities
    const T* G;         // n_i^d  w_j g_j (the nodal factor of every triple)
    const T* sym;       // np^d orbit sums, p_1 fastest (slab scheme)
    const int* pair_a;  // np  smaller node of each pair
    const int* pair_b;  // np  larger node
    const int* pair_base;  // n_i  index of the pair (a, a)
    const T* sigma;     // n_sigma x d
    const T* wfac;      // n_sigma  W_s b0 S^d, formed in FP64 and rounded once
    const T* poly;      // terms x W  (slab scheme)
    const double* poly64;  // terms x W  the same coefficients in FP64 (binned schemes)
    const double* kpoly_eo;  // even and odd parts of the cells a < W/2 (binned scheme)
    const double* cellfit;   // per bin coordinate: w_c, 1/delta and the offset polynomial
    const double* cellfit_v; // per bin coordinate: t_c, 1/delta (0: none), offset and map-factor polynomials in v/S
    const T* slab_vlo;  // n_slabs
    const T* slab_vhi;
    double* partial;    // n_chunks x n_g^d
    T S, inv_S, h_inv, b0, gamma;
    T aniso;            // beta of the angle-dependent rate b0 |u|^gamma (1 + beta cos^2 theta)
    double inv_S64, h_inv64;  // 1/S and 1/h in FP64
    int map, vhs, ni, np, ng, nh, slab_planes, n_sigma;  // vhs: the rate carries |u|^gamma
    int64_t ngd, n_units, units_per_chunk;
};

// post-collision coordinate in the transform variable and the factor mu^-2 / S
// (the constant S of every dimension sits in the direction weight wfac):
//   r = 0: zeta = tanh(t), z = arccos zeta = 2 atan(exp(-t)), mu^-2 / S = cosh(t)
//   r = 1: zeta = t/sqrt(1+t^2), z = atan2(1, t),             mu^-2 / S = 1 + t^2
// with t = v/S.  Evaluated in FP64 for both precisions: the FP32 exp and atan
// of the device library carry a small bias that moves every point the same
// way, which left a floor of about 4e-7 (relative) in an FP32 gain, while
// these few FP64 operations per point cost little next to the spreading.
template <typename T>
__device__ __forceinline__ void map_point(T v, const GainParams<T>& P, double& z, T& m2)
{
    const double t = (double)v * P.inv_S64;
    if (P.map == 0) {
        const double e = exp(-t);
        z = 2.0 * atan(e);
        m2 = (T)(0.5 * (e + 1.0 / e));
    } else {
        z = atan2(1.0, t);
        m2 = (T)fma(t, t, 1.0);
    }
}

// 1/x for positive normal x: the hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Both maps send a velocity to the transform angle as z = pi/2 - 2 atan(w) with
// w in (-1, 1):
//   r = 0: w = tanh(t/2) = (1 - e^-t) / (1 + e^-t),  mu^-2 / S = cosh t
//   r = 1: w = t / (1 + sqrt(1 + t^2)),               mu^-2 / S = 1 + t^2
// (t = v/S).  Returns w; the arctangent itself is never formed: inside one grid
// cell the kernel offset is a short polynomial in w (cell_offset).
template <typename T>
__device__ __forceinline__ double map_w(T v, const GainParams<T>& P, T& m2)
{
    const double t = (double)v * P.inv_S64;
    if (P.map == 0) {
        // one reciprocal for both: with R = 1 / (e (1 + e)), 1/e = (1 + e) R and
        // 1/(1 + e) = e R
        const double e = exp(-t);
        const double ep = 1.0 + e;
        const double R = rcp64(e * ep);
        m2 = (T)(0.5 * fma(ep, R, e));
        return (1.0 - e) * (e * R);
    }
    const double r = fma(t, t, 1.0);
    m2 = (T)r;
    return t * rcp64(1.0 + sqrt(r));
}

// sum_k c[k] x^k (k = 0 .. DEG) by Horner's rule, for coefficients that are
// the same on every lane (scalar registers).  The sum is carried negated,
// u <- u x - c[k]: each step is then one three-operand FMA with the scalar
// coefficient negated in place, where the plain form makes the compiler copy
// every coefficient into a vector register first to use the two-operand FMA.
// Negation is exact, so the result equals the plain Horner sum bit for bit.
template <int DEG>
__device__ __forceinline__ double horner_uniform(const double* __restrict__ c, double x)
{
    double u = -c[DEG];
#pragma unroll
    for (int k = DEG - 1; k >= 0; --k) u = fma(u, x, -c[k]);
    return -u;
}

// kernel offset s = 2 (t0 - z/h + W/2) - 1 of a point whose footprint corner
// in this dimension is t0, from the fit of that cell
__device__ __forceinline__ double cell_offset(const double* __restrict__ cf, double w)
{
    const double x = (w - cf[0]) * cf[1];
    return horner_uniform<kCellFitDeg>(cf + 2, x);
}

// kernel offset and map factor m2 of a point from its cell's fit in the scaled
// velocity t = v/S (a cell with a nonzero 1/delta in cv[1]); FP32 plans hold
// fits of a lower degree in the same slots
template <typename T>
__device__ __forceinline__ double cell_offset_v(const double* __restrict__ cv, T v, double inv_S64, T& m2)
{
    constexpr int DEG = sizeof(T) == sizeof(double) ? kCellFitDeg : kCellFitDegV32;
    const double x = ((double)v * inv_S64 - cv[0]) * cv[1];
    m2 = (T)horner_uniform<DEG>(cv + 3 + kCellFitDeg, x);
    return horner_uniform<DEG>(cv + 2, x);
}

// values of the W kernel cells at offset s in [-1, 1): Horner in s
template <typename T, int W, int TERMS>
__device__ __forceinline__ void kernel_cells(const T* __restrict__ poly, T s, T* out)
{
#pragma unroll
    for (int a = 0; a < W; ++a) out[a] = poly[(TERMS - 1) * W + a];
#pragma unroll
    for (int d = TERMS - 2; d >= 0; --d) {
#pragma unroll
        for (int a = 0; a < W; ++a) out[a] = fma(out[a], s, poly[d * W + a]);
    }
}

// The same kernel values from the FP64 coefficients, evaluated in FP64 and
// rounded once to T.  The monomial coefficients of the cells are several
// times larger than the kernel values, so FP32 coefficients and an FP32 Horner
// sweep would leave a systematic error of a few 1e-7 in every kernel value,
// which the deconvolution by the exact kernel transform does not undo.  A
// gfx950 lane issues an FP64 FMA at the rate of an FP32 one.
template <typename T, int W, int TERMS>
__device__ __forceinline__ void kernel_cells64(const double* __restrict__ poly, double s, T* out)
{
    double v[W];
#pragma unroll
    for (int a = 0; a < W; ++a) v[a] = poly[(TERMS - 1) * W + a];
#pragma unroll
    for (int d = TERMS - 2; d >= 0; --d) {
#pragma unroll
        for (int a = 0; a < W; ++a) v[a] = fma(v[a], s, poly[d * W + a]);
    }
#pragma unroll
    for (int a = 0; a < W; ++a) out[a] = (T)v[a];
}

// The same values from the mirror symmetry of the cells: cell W-1-a at s is
// cell a at -s, so with u = s^2 and the even and odd parts E_a(u), O_a(u) of
// cell a (a < W/2) the pair is E_a + s O_a and E_a - s O_a; a middle cell is
// even.  Layout: even parts [TERMS+1 / 2][(W+1)/2], then odd parts [TERMS/2][W/2].
template <typename T, int W, int TERMS>
__device__ __forceinline__ void kernel_cells_eo(const double* __restrict__ eo, double s, T* out)
{
    constexpr int H = (W + 1) / 2, HP = W / 2;
    constexpr int NE = (TERMS + 1) / 2, NO = TERMS / 2;
    const double* ev = eo;
    const double* od = eo + NE * H;
    const double u = s * s;
    double e[H], o[HP];
#pragma unroll
    for (int a = 0; a < H; ++a) e[a] = ev[(NE - 1) * H + a];
#pragma unroll
    for (int j = NE - 2; j >= 0; --j) {
#pragma unroll
        for (int a = 0; a < H; ++a) e[a] = fma(e[a], u, ev[j * H + a]);
    }
#pragma unroll
    for (int a = 0; a < HP; ++a) o[a] = od[(NO - 1) * HP + a];
#pragma unroll
    for (int j = NO - 2; j >= 0; --j) {
#pragma unroll
        for (int a = 0; a < HP; ++a) o[a] = fma(o[a], u, od[j * HP + a]);
    }
#pragma unroll
    for (int a = 0; a < HP; ++a) {
        out[a] = (T)fma(s, o[a], e[a]);
        out[W - 1 - a] = (T)fma(-s, o[a], e[a]);
    }
    if constexpr ((W & 1) != 0) out[H - 1] = (T)e[H - 1];
}

// kernel_cells_eo for the DIM offsets of one point at once, cell pair by cell
// pair: each coefficient is loaded once (a scalar load: the table is the same
// for every lane) and used DIM times, so few coefficients are live at a time.
// Every value goes to sink(l, a, value) as soon as it is formed.
template <typename T, int W, int TERMS, int DIM, typename Sink>
__device__ __forceinline__ void kernel_cells_eo_each(const double* __restrict__ eo, const double* sv, Sink&& sink)
{
    constexpr int H = (W + 1) / 2, HP = W / 2;
    constexpr int NE = (TERMS + 1) / 2, NO = TERMS / 2;
    const double* ev = eo;
    const double* od = eo + NE * H;
    double u[DIM];
#pragma unroll
    for (int l = 0; l < DIM; ++l) u[l] = sv[l] * sv[l];
#pragma unroll
    for (int a = 0; a < H; ++a) {
        double e[DIM], o[DIM];
        const double ce = ev[(NE - 1) * H + a];
#pragma unroll
        for (int l = 0; l < DIM; ++l) e[l] = ce;
#pragma unroll
        for (int j = NE - 2; j >= 0; --j) {
            const double c = ev[j * H + a];
#pragma unroll
            for (int l = 0; l < DIM; ++l) e[l] = fma(e[l], u[l], c);
        }
        if (a < HP) {
            const double co = od[(NO - 1) * HP + a];
#pragma unroll
            for (int l = 0; l < DIM; ++l) o[l] = co;
#pragma unroll
            for (int j = NO - 2; j >= 0; --j) {
                const double c = od[j * HP + a];
#pragma unroll
                for (int l = 0; l < DIM; ++l) o[l] = fma(o[l], u[l], c);
            }
#pragma unroll
            for (int l = 0; l < DIM; ++l) {
                sink(l, a, (T)fma(sv[l], o[l], e[l]));
                sink(l, W - 1 - a, (T)fma(-sv[l], o[l], e[l]));
            }
        } else {
#pragma unroll
            for (int l = 0; l < DIM; ++l) sink(l, a, (T)e[l]);
        }
    }
}

// the same into an array out[l][a]
template <typename T, int W, int TERMS, int DIM>
__device__ __forceinline__ void kernel_cells_eo_dims(const double* __restrict__ eo, const double* sv,
                                                     T (*out)[W])
{
    kernel_cells_eo_each<T, W, TERMS, DIM>(eo, sv, [&](int l, int a, T v) { out[l][a] = v; });
}

// base[i] for a table of fewer than 2^32 bytes: a 32-bit byte offset from a
// base that is the same on every lane, which the loads take in their
// scalar-base form (no per-lane 64-bit address arithmetic)
template <typename T>
__device__ __forceinline__ T ld_u32(const T* __restrict__ base, unsigned i)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}

// The node pair (a_l <= b_l) of every dimension of one merged point.
template <int DIM>
struct PairNodes {
    int a[DIM], b[DIM];
};

// the node pairs of a merged point given by the pair indices p_2, p_3 of the
// later dimensions (the pair tables list the unordered pairs)
template <typename T, int DIM>
__device__ __forceinline__ PairNodes<DIM> pair_nodes(const GainParams<T>& P, int a1, int b1, int p2, int p3)
{
    PairNodes<DIM> nd;
    nd.a[0] = a1;
    nd.b[0] = b1;
    nd.a[1] = P.pair_a[p2];
    nd.b[1] = P.pair_b[p2];
    if constexpr (DIM == 3) {
        nd.a[2] = P.pair_a[p3];
        nd.b[2] = P.pair_b[p3];
    }
    return nd;
}

// Merged point ids pack the direction s and the nodes of every dimension as
// b1 | a1 << 8 | s << 16 | a2 << 26 | b2 << 34 | a3 << 42 | b3 << 50 (58 bits;
// 256 interior nodes per dimension and 1024 directions at most).  Carrying the
// nodes, not the pair indices, lets the spreading kernels fetch the node
// velocities and nodal values of a point in one round of loads.
template <int DIM>
__device__ __forceinline__ unsigned long long pack_id(int s, const PairNodes<DIM>& nd)
{
    unsigned long long id = (unsigned long long)nd.b[0] | ((unsigned long long)nd.a[0] << 8) |
                            ((unsigned long long)s << 16) | ((unsigned long long)nd.a[1] << 26) |
                            ((unsigned long long)nd.b[1] << 34);
    if constexpr (DIM == 3) id |= ((unsigned long long)nd.a[2] << 42) | ((unsigned long long)nd.b[2] << 50);
    return id;
}

template <int DIM>
__device__ __forceinline__ PairNodes<DIM> unpack_id(unsigned long long id, int& s)
{
    PairNodes<DIM> nd;
    nd.b[0] = (int)(id & 0xffull);
    nd.a[0] = (int)((id >> 8) & 0xffull);
    s = (int)((id >> 16) & 0x3ffull);
    nd.a[1] = (int)((id >> 26) & 0xffull);
    nd.b[1] = (int)((id >> 34) & 0xffull);
    if constexpr (DIM == 3) {
        nd.a[2] = (int)((id >> 42) & 0xffull);
        nd.b[2] = (int)((id >> 50) & 0xffull);
    }
    return nd;
}

// post-collision velocity of one merged point and its weight without the map
// factors and the orbit sum: q = W_s b0 S^d (times |u|^gamma for VHS)
template <typename T, int DIM>
__device__ __forceinline__ void point_velocity(const GainParams<T>& P, int s, const PairNodes<DIM>& nd, T& q,
                                               T* vp)
{
    const T half = (T)0.5;
    T r2 = (T)0;
#pragma unroll
    for (int l = 1; l < DIM; ++l) {
        const T x = ld_u32(P.v1, nd.a[l]), y = ld_u32(P.v1, nd.b[l]);
        vp[l] = (x + y) * half;
        r2 += (x - y) * (x - y);
    }
    // |u|^2 summed as d_1^2 + (d_2^2 + d_3^2), as the slab scheme sums it
    const T va = ld_u32(P.v1, nd.a[0]), vb = ld_u32(P.v1, nd.b[0]);
    const T d = va - vb;
    const T un = sqrt(d * d + r2);
    vp[0] = (va + vb) * half + un * ld_u32(P.sigma, s * DIM) * half;
#pragma unroll
    for (int l = 1; l < DIM; ++l) vp[l] += un * ld_u32(P.sigma, s * DIM + l) * half;
    q = ld_u32(P.wfac, s);
    if (P.vhs) q *= (P.gamma == (T)1) ? un : (un > (T)0 ? pow(un, P.gamma) : (T)(P.gamma == (T)0));
}

// geometry of one merged point: weight without the orbit sum, and z/h - W/2
// (in FP64 from z, so that bins and kernel offsets agree for both precisions)
template <typename T, int DIM>
__device__ __forceinline__ void point_geometry(const GainParams<T>& P, int s, const PairNodes<DIM>& nd,
                                               double halfW, T& q, double* xs)
{
    T vp[DIM];
    point_velocity<T, DIM>(P, s, nd, q, vp);
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
        double z;
        T m2;
        map_point(vp[l], P, z, m2);
        q *= m2;
        xs[l] = z * P.h_inv64 - halfW;
    }
}

// The 2^(d-1) products G_x G_y of the orbit of one merged point: the 2^d
// exchanges of (a_l, b_l) pair up into products counted twice, and each equal
// pair a_l = b_l halves the count.  Writes the flat node indices of the
// products and returns the multiplicity c.
template <typename T, int DIM>
__device__ __forceinline__ T orbit_terms(const GainParams<T>& P, const PairNodes<DIM>& nd, int* ix, int* iy)
{
    const int ni = P.ni;
    const int a1 = nd.a[0], b1 = nd.b[0], a2 = nd.a[1], b2 = nd.b[1];
    T c = (T)2;
    if (a1 == b1) c *= (T)0.5;
    if (a2 == b2) c *= (T)0.5;
    if constexpr (DIM == 2) {
        ix[0] = a1 * ni + a2;
        iy[0] = b1 * ni + b2;
        ix[1] = a1 * ni + b2;
        iy[1] = b1 * ni + a2;
    } else {
        const int a3 = nd.a[2], b3 = nd.b[2];
        if (a3 == b3) c *= (T)0.5;
        const int A1 = a1 * ni, B1 = b1 * ni;
        ix[0] = (A1 + a2) * ni + a3;
        iy[0] = (B1 + b2) * ni + b3;
        ix[1] = (A1 + a2) * ni + b3;
        iy[1] = (B1 + b2) * ni + a3;
        ix[2] = (A1 + b2) * ni + a3;
        iy[2] = (B1 + a2) * ni + b3;
        ix[3] = (A1 + b2) * ni + b3;
        iy[3] = (B1 + a2) * ni + a3;
    }
    return c;
}

// Orbit sum of one merged point straight from the nodal table G (small enough
// to stay in L2).
template <typename T, int DIM>
__device__ __forceinline__ T orbit_sum(const GainParams<T>& P, const PairNodes<DIM>& nd)
{
    constexpr int NT = 1 << (DIM - 1);
    int ix[NT], iy[NT];
    const T c = orbit_terms<T, DIM>(P, nd, ix, iy);
    T acc = ld_u32(P.G, ix[0]) * ld_u32(P.G, iy[0]);
#pragma unroll
    for (int t = 1; t < NT; ++t) acc = fma(ld_u32(P.G, ix[t]), ld_u32(P.G, iy[t]), acc);
    return c * acc;
}

// The orbit sum of an angle-dependent rate B = R(|u|) (1 + beta cos^2 theta),
// cos theta = u.sigma_s / |u|.  The triples of one orbit share |u| but not the
// angle: exchanging i_l and j_l flips u_l.  Term t of orbit_terms takes node a
// of the first dimension for i and flips the dimensions where it takes b, so
// its cos theta is sum_l eps_l e_l / |u| with e_l = (v_{a_l} - v_{b_l}) sigma_l;
// the mirror triple (i and j exchanged) flips every sign and keeps cos^2, which
// is what the multiplicity 2 of each term counts.  u = 0 gives cos theta = 0.
template <typename T, int DIM>
__device__ __forceinline__ T orbit_sum_aniso(const GainParams<T>& P, int s, const PairNodes<DIM>& nd)
{
    constexpr int NT = 1 << (DIM - 1);
    int ix[NT], iy[NT];
    const T c = orbit_terms<T, DIM>(P, nd, ix, iy);
    T e[DIM], u2 = (T)0;
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
        const T dl = P.v1[nd.a[l]] - P.v1[nd.b[l]];
        u2 += dl * dl;
        e[l] = dl * P.sigma[s * DIM + l];
    }
    const T k = u2 > (T)0 ? P.aniso / u2 : (T)0;
    T acc = (T)0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        // 2D: t = 0 (+, +), 1 (+, -); 3D: t = 0 (+, +, +), 1 (+, +, -), 2 (+, -, +), 3 (+, -, -)
        T proj = e[0];
        if constexpr (DIM == 2) proj += (t & 1) ? -e[1] : e[1];
        else proj += ((t & 2) ? -e[1] : e[1]) + ((t & 1) ? -e[2] : e[2]);
        acc = fma(P.G[ix[t]] * P.G[iy[t]], fma(k * proj, proj, (T)1), acc);
    }
    return c * acc;
}

struct BinGeo {
    int nb;      // bins per dimension
    int off;     // bin index = t0 + off
    int W;
    int64_t n_items;  // (s, a_1, pencil) generation items
    int s0, ns;       // directions [s0, s0 + ns) of the generation items
    unsigned long long id_cap;  // scatter: ids the buffer holds (no write at or past it)
    const double* vthr;         // nb + 2 velocity thresholds V_k, k = -off - 1 ..
    float h_inv, half_w;        // 1/h and W/2 for the FP32 estimate
};

// Bin coordinate of one velocity component: the smallest k with v >= V_k
// (V decreasing), then k + off clamped to the bins.  An FP32 evaluation of the
// transform angle places k to within one of the answer, and two FP64
// comparisons with the table settle it.  A velocity within 1e-9 S of the
// deciding threshold (symmetric node pairs put many points exactly on a cell
// boundary) takes ceil(z/h - W/2) of the FP64 angle instead, as the slab
// scheme does: at a boundary both footprints are valid and differ by the
// kernel's edge value, so every scheme must pick the same one.
template <typename T>
__device__ __forceinline__ int bin_coord(double v, const GainParams<T>& P, const BinGeo& B)
{
    const float t = (float)(v * P.inv_S64);
    const float z = P.map == 0 ? 2.0f * atanf(expf(-t)) : atan2f(1.0f, t);
    int k = (int)ceilf(z * B.h_inv - B.half_w);
    const int kmin = -B.off - 1, kmax = B.nb - B.off;  // the table's k range
    k = k < kmin + 1 ? kmin + 1 : (k > kmax - 1 ? kmax - 1 : k);
    const double* V = B.vthr - kmin;
    const double lo = V[k - 1], hi = V[k];
    const bool above_lo = v >= lo, above_hi = v >= hi;
    const double near = above_lo ? v - lo : (above_hi ? fmin(v - hi, lo - v) : hi - v);
    if (near <= 1e-9 / P.inv_S64) {
        double zz;
        T m2;
        map_point((T)v, P, zz, m2);
        k = (int)ceil(zz * P.h_inv64 - 0.5 * B.W);
    } else {
        k = above_lo ? k - 1 : (above_hi ? k : k + 1);
    }
    const int c = k + B.off;
    return c < 0 ? 0 : (c >= B.nb ? B.nb - 1 : c);
}

}  // namespace
}  // namespace pgc
