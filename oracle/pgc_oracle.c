/*
 * pgc_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see the
 * header).  Every sum here is written out as the paper defines it, with no
 * blocking, no fast transform and no NUFFT: the gain and loss are the
 * Chebyshev-Gauss-Lobatto discretisations of eqs. (Qplus) and (Qminus) of
 * Sec. 4.2, summed directly over the collision triples (sigma_s, xi_i, eta_j).
 *
 * Readings taken where the paper is silent:
 *   - every velocity sum runs over the interior CGL nodes; f_N = mu^4 P and
 *     f_N / mu^2 vanish at xi = +-1 (v = +-inf), so the endpoints drop out of
 *     the gain exactly and out of the loss up to a term of size P(+-1);
 *   - mu(zeta)^-2 and 1 - zeta^2 are evaluated from v' itself
 *     (S cosh(v'/S) for r = 0, (S^2 + v'^2)/S for r = 1), which equals the
 *     paper's expression in zeta and avoids cancellation as zeta -> +-1.
 */
#include "pgc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846264338327950288

/* c_0 = pi, c_k = pi/2: the Chebyshev norms (T_k, T_k)_omega, Sec. 2.1. */
static double cheb_norm(int k) { return k == 0 ? ORA_PI : 0.5 * ORA_PI; }

/* v(xi) for the logarithmic (r = 0) and algebraic (r = 1) maps, Sec. 2.1. */
static double map_v(int map, double S, double xi)
{
    if (map == 0) return S * atanh(xi);
    return S * xi / sqrt(1.0 - xi * xi);
}

/* xi(v), the inverse maps of Sec. 2.1. */
static double map_xi(int map, double S, double v)
{
    if (map == 0) return tanh(v / S);
    return v / sqrt(S * S + v * v);
}

/* mu(xi)^2 = (1 - xi^2)^{(1+r)/2} / S, eq. (1D_mu_function). */
static double mu2_of_xi(int map, double S, double xi)
{
    double s = 1.0 - xi * xi;
    return (map == 0 ? sqrt(s) : s) / S;
}

/* mu(xi(v))^-2 written in v: 1 - tanh^2 = sech^2 for r = 0 and
 * 1 - v^2/(S^2+v^2) = S^2/(S^2+v^2) for r = 1. */
static double inv_mu2_of_v(int map, double S, double v)
{
    if (map == 0) return S * cosh(v / S);
    return (S * S + v * v) / S;
}

/* zeta = xi(v') and mu(zeta)^-2 together; for r = 0 both come from one
 * exponential, e = exp(v/S): tanh = (e - 1/e)/(e + 1/e), S cosh = S (e + 1/e)/2. */
static void test_point(int map, double S, double v, double* zeta, double* m2)
{
    if (map == 0) {
        double e = exp(v / S), ei = 1.0 / e;
        *zeta = (e - ei) / (e + ei);
        *m2 = 0.5 * S * (e + ei);
    } else {
        *zeta = map_xi(map, S, v);
        *m2 = inv_mu2_of_v(map, S, v);
    }
}

/* mu(xi(v))^4 written in v, the weight of the trial functions T~_k. */
static double mu4_of_v(int map, double S, double v)
{
    if (map == 0) {
        double c = cosh(v / S);
        return 1.0 / (c * c * S * S);
    }
    double d = S * S + v * v;
    return S * S / (d * d);
}

/* T_k(x)/sqrt(c_k) for k = 0..n-1 by the three-term recurrence of Sec. 2.1
 * (1/sqrt(c_k) is 1/sqrt(pi) for k = 0 and sqrt(2/pi) otherwise). */
static void cheb_scaled(double x, int n, double* out)
{
    const double r0 = 1.0 / sqrt(cheb_norm(0)), r1 = 1.0 / sqrt(cheb_norm(1));
    double tm = 1.0, t = x;
    if (n > 0) out[0] = r0;
    if (n > 1) out[1] = x * r1;
    for (int k = 2; k < n; ++k) {
        const double tk = 2.0 * x * t - tm;
        tm = t;
        t = tk;
        out[k] = tk * r1;
    }
}

static int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

/* digits of a flat row-major index, last dimension fastest */
static void unflat(int64_t f, int dim, int64_t n, int* idx)
{
    for (int l = dim - 1; l >= 0; --l) {
        idx[l] = (int)(f % n);
        f /= n;
    }
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int ora_cgl(int m_v, int map, double S, double* xi, double* v, double* w, double* mu2)
{
    if (m_v < 3 || S <= 0.0 || (map != 0 && map != 1)) return -1;
    for (int j = 0; j < m_v; ++j) {
        double x = -cos(ORA_PI * j / (m_v - 1));
        int end = (j == 0 || j == m_v - 1);
        if (j == 0) x = -1.0;
        if (j == m_v - 1) x = 1.0;
        if (xi) xi[j] = x;
        if (w) w[j] = end ? ORA_PI / (2.0 * (m_v - 1)) : ORA_PI / (m_v - 1);
        if (v) v[j] = end ? (j == 0 ? -HUGE_VAL : HUGE_VAL) : map_v(map, S, x);
        if (mu2) mu2[j] = end ? 0.0 : mu2_of_xi(map, S, x);
    }
    return 0;
}

int ora_circle_rule(int m, double* sigma, double* w)
{
    if (m < 1) return -1;
    for (int s = 0; s < m; ++s) {
        double th = 2.0 * ORA_PI * s / m;
        sigma[2 * s] = cos(th);
        sigma[2 * s + 1] = sin(th);
        w[s] = 2.0 * ORA_PI / m;
    }
    return 0;
}

int ora_gauss_legendre(int n, double* x, double* w)
{
    if (n < 1) return -1;
    for (int i = 0; i < n; ++i) {
        /* Newton on P_n from the Chebyshev-like first guess */
        double t = cos(ORA_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
        }
        x[n - 1 - i] = t;
        w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    return 0;
}

int ora_sphere_product_rule(int n_t, int n_p, double* sigma, double* w)
{
    if (n_t < 1 || n_p < 1) return -1;
    double* x = (double*)malloc(sizeof(double) * n_t);
    double* wx = (double*)malloc(sizeof(double) * n_t);
    ora_gauss_legendre(n_t, x, wx);
    int s = 0;
    for (int a = 0; a < n_t; ++a) {
        double st = sqrt(1.0 - x[a] * x[a]);
        for (int b = 0; b < n_p; ++b, ++s) {
            double ph = 2.0 * ORA_PI * b / n_p;
            sigma[3 * s] = st * cos(ph);
            sigma[3 * s + 1] = st * sin(ph);
            sigma[3 * s + 2] = x[a];
            w[s] = wx[a] * 2.0 * ORA_PI / n_p;
        }
    }
    free(x);
    free(wx);
    return 0;
}

/* ---- shared set-up for one problem: interior node tables ---------------- */

typedef struct {
    int dim, N, ni;
    int64_t nd, Nd;
    double* v1;   /* ni        mapped interior nodes */
    double* w1;   /* ni        CGL weights */
    double* mu21; /* ni        mu(xi)^2 */
    double* tn;   /* ni x N    T_k(xi_a)/sqrt(c_k) */
} ora_tables;

static int check_problem(const ora_problem* p)
{
    if (!p || (p->dim != 2 && p->dim != 3) || p->n_modes < 1 || p->m_v < 3 ||
        p->S <= 0.0 || (p->map != 0 && p->map != 1) || p->kernel < 0 || p->kernel > 2 ||
        (p->kernel == 2 && !(p->aniso >= -1.0 && p->aniso <= 10.0)))
        return -1;
    return 0;
}

static void tables_init(const ora_problem* p, ora_tables* t)
{
    int m = p->m_v;
    t->dim = p->dim;
    t->N = p->n_modes;
    t->ni = m - 2;
    t->nd = ipow(t->ni, p->dim);
    t->Nd = ipow(t->N, p->dim);
    double* xi = (double*)malloc(sizeof(double) * m);
    double* v = (double*)malloc(sizeof(double) * m);
    double* w = (double*)malloc(sizeof(double) * m);
    double* mu2 = (double*)malloc(sizeof(double) * m);
    ora_cgl(m, p->map, p->S, xi, v, w, mu2);
    t->v1 = (double*)malloc(sizeof(double) * t->ni);
    t->w1 = (double*)malloc(sizeof(double) * t->ni);
    t->mu21 = (double*)malloc(sizeof(double) * t->ni);
    t->tn = (double*)malloc(sizeof(double) * t->ni * t->N);
    for (int a = 0; a < t->ni; ++a) {
        t->v1[a] = v[a + 1];
        t->w1[a] = w[a + 1];
        t->mu21[a] = mu2[a + 1];
        cheb_scaled(xi[a + 1], t->N, t->tn + (size_t)a * t->N);
    }
    free(xi);
    free(v);
    free(w);
    free(mu2);
}

static void tables_free(ora_tables* t)
{
    free(t->v1);
    free(t->w1);
    free(t->mu21);
    free(t->tn);
}

/* sum over all k of c[k] prod_l M[i_l][k_l] for a node multi-index i */
static void nodal_values(const ora_tables* t, const double* coeffs, double* P)
{
    int dim = t->dim, N = t->N;
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < t->nd; ++f) {
        int ii[3];
        unflat(f, dim, t->ni, ii);
        double s = 0.0;
        for (int64_t k = 0; k < t->Nd; ++k) {
            int kk[3];
            unflat(k, dim, N, kk);
            double b = coeffs[k];
            for (int l = 0; l < dim; ++l) b *= t->tn[(size_t)ii[l] * N + kk[l]];
            s += b;
        }
        P[f] = s;
    }
}

int ora_nodal(const ora_problem* p, const double* coeffs, double* P_int)
{
    if (check_problem(p)) return -1;
    ora_tables t;
    tables_init(p, &t);
    nodal_values(&t, coeffs, P_int);
    tables_free(&t);
    return 0;
}

/* f_k = (f, T^_k) by the CGL rule on the interior nodes: eq.
 * (MultiD_spectral_coef), f~_k = c_k^{-1/2} (mu^-4 f, T_k)_omega. */
int ora_project(const ora_problem* p, const double* f_int, double* coeffs)
{
    if (check_problem(p)) return -1;
    ora_tables t;
    tables_init(p, &t);
    int dim = t.dim, N = t.N;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < t.Nd; ++k) {
        int kk[3];
        unflat(k, dim, N, kk);
        double s = 0.0;
        for (int64_t f = 0; f < t.nd; ++f) {
            int ii[3];
            unflat(f, dim, t.ni, ii);
            double b = f_int[f];
            for (int l = 0; l < dim; ++l) {
                double m2 = t.mu21[ii[l]];
                b *= t.w1[ii[l]] / (m2 * m2) * t.tn[(size_t)ii[l] * N + kk[l]];
            }
            s += b;
        }
        coeffs[k] = s;
    }
    tables_free(&t);
    return 0;
}

/* B(|u|, cos theta), u = v - v_*, cos theta = u.sigma/|u| (0 when u = 0).
 * Maxwell (b0) and VHS (b0 |u|^gamma) do not depend on the angle; kernel 2
 * weights the VHS rate by 1 + aniso cos^2 theta.  Q(f, f) sees only the part
 * of B that is even in cos theta (relabelling v and v_* flips its sign), and
 * an even polynomial keeps B smooth where cos theta = -1 or 1. */
static double kernel_b(const ora_problem* p, double un, double c)
{
    if (p->kernel == 0) return p->b0;
    double b = un == 0.0 ? (p->gamma == 0.0 ? p->b0 : 0.0) : p->b0 * pow(un, p->gamma);
    if (p->kernel == 2) b *= 1.0 + p->aniso * c * c;
    return b;
}

static double cos_theta(const double* vi, const double* vj, const double* sg, int dim, double un)
{
    if (un == 0.0) return 0.0;
    double d = 0.0;
    for (int l = 0; l < dim; ++l) d += (vi[l] - vj[l]) * sg[l];
    return d / un;
}

/* Per-node data: v_i (dim), w_i g_i where g = f_N / mu^2 = mu^2 P, and P_i. */
typedef struct {
    double* v;  /* nd x dim */
    double* wg; /* nd */
    double* P;  /* nd */
    double* w;  /* nd */
} ora_nodes;

static void nodes_init(const ora_tables* t, const double* coeffs, ora_nodes* nd)
{
    int dim = t->dim;
    nd->v = (double*)malloc(sizeof(double) * t->nd * dim);
    nd->wg = (double*)malloc(sizeof(double) * t->nd);
    nd->P = (double*)malloc(sizeof(double) * t->nd);
    nd->w = (double*)malloc(sizeof(double) * t->nd);
    nodal_values(t, coeffs, nd->P);
    for (int64_t f = 0; f < t->nd; ++f) {
        int ii[3];
        unflat(f, dim, t->ni, ii);
        double w = 1.0, mu2 = 1.0;
        for (int l = 0; l < dim; ++l) {
            nd->v[f * dim + l] = t->v1[ii[l]];
            w *= t->w1[ii[l]];
            mu2 *= t->mu21[ii[l]];
        }
        nd->w[f] = w;
        nd->wg[f] = w * mu2 * nd->P[f];
    }
}

static void nodes_free(ora_nodes* nd)
{
    free(nd->v);
    free(nd->wg);
    free(nd->P);
    free(nd->w);
}

/* The loss, eq. (Qminus) discretised: A_i = sum_s W_s sum_j w_j g_j B(|v_i - v_j|, cos theta)
 * is the inner integral, and Q-_k = sum_i w_i A_i f_N(v_i) T^_k(v_i) / mu_i^2
 * = sum_i w_i A_i P_i T_k(xi_i)/sqrt(c_k) is the outer one. */
static void loss_field(const ora_problem* p, const ora_tables* t, const ora_nodes* nd, double* A)
{
    int dim = t->dim;
    double wsum = 0.0;
    for (int s = 0; s < p->n_sigma; ++s) wsum += p->sigma_w[s];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < t->nd; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < t->nd; ++j) {
            const double* vi = nd->v + i * dim;
            const double* vj = nd->v + j * dim;
            double un2 = 0.0;
            for (int l = 0; l < dim; ++l) un2 += (vi[l] - vj[l]) * (vi[l] - vj[l]);
            const double un = sqrt(un2);
            if (p->kernel == 2) {
                /* an angle-dependent rate: the inner integral over sigma itself */
                for (int s = 0; s < p->n_sigma; ++s)
                    acc += p->sigma_w[s] * nd->wg[j] *
                           kernel_b(p, un, cos_theta(vi, vj, p->sigma + (size_t)s * dim, dim, un));
            } else {
                acc += nd->wg[j] * kernel_b(p, un, 0.0);
            }
        }
        A[i] = p->kernel == 2 ? acc : wsum * acc;
    }
}

/* Compensated accumulation (Ogita, Rump and Oishi, "Accurate sum and dot
 * product", SIAM J. Sci. Comput. 26 (2005), algorithm Sum2): the rounding error
 * of each addition s + x is recovered exactly by Knuth's TwoSum and collected
 * in c, so s + c carries the sum as if it were formed in twice the working
 * precision.  The gain of one coefficient adds up to n_sigma * n_i^(2 dim)
 * terms (5e8 for a 2D 64-mode problem), whose plain sequential sum would lose
 * about 1e-11 relative: more than the error of the method being checked. */
static inline void sum2_add(double* s, double* c, double x)
{
    const double t = *s + x;
    const double bp = t - *s;
    *c += (*s - (t - bp)) + (x - bp);
    *s = t;
}

/* The gain, eq. (Qplus) with (Qplus1), (FF) and (num_fast_k) before any fast
 * transform: for every triple (s, i, j)
 *   v' = (v_i + v_j)/2 + |v_i - v_j| sigma_s / 2,
 *   weight = W_s w_i g_i w_j g_j B(|v_i - v_j|),
 *   Q+_k += weight * T^_k(v'),  T^_k(v') = prod_l mu(zeta_l)^-2 T_{k_l}(zeta_l)/sqrt(c_{k_l}).
 * Units (s, i) are split statically over threads; every addition is
 * compensated (sum2_add) and the per-thread partial sums are added in thread
 * order.  With n_k > 0 only the listed k are formed. */
static void gain_sum(const ora_problem* p, const ora_tables* t, const ora_nodes* nd,
                     int n_k, const int* kidx, int64_t u_lo, int64_t u_hi, double* out)
{
    int dim = t->dim, N = t->N;
    int64_t nout = n_k > 0 ? n_k : t->Nd;
    int nth = ora_num_threads();
    /* per thread: nout running sums followed by nout compensations */
    double* part = (double*)calloc((size_t)nth * 2 * nout, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* acc = part + (size_t)tid * 2 * nout;
        double* cmp = acc + nout;
        double* a = (double*)malloc(sizeof(double) * 3 * N);
#pragma omp for schedule(static)
        for (int64_t u = u_lo; u < u_hi; ++u) {
            int s = (int)(u / t->nd);
            int64_t i = u % t->nd;
            const double* sg = p->sigma + (size_t)s * dim;
            const double* vi = nd->v + i * dim;
            double wi = p->sigma_w[s] * nd->wg[i];
            if (wi == 0.0) continue;
            for (int64_t j = 0; j < t->nd; ++j) {
                const double* vj = nd->v + j * dim;
                double un2 = 0.0;
                for (int l = 0; l < dim; ++l) un2 += (vi[l] - vj[l]) * (vi[l] - vj[l]);
                double un = sqrt(un2);
                double wt = wi * nd->wg[j] * kernel_b(p, un, cos_theta(vi, vj, sg, dim, un));
                if (wt == 0.0) continue;
                for (int l = 0; l < dim; ++l) {
                    double vp = 0.5 * (vi[l] + vj[l]) + 0.5 * un * sg[l];
                    double zeta, m2;
                    test_point(p->map, p->S, vp, &zeta, &m2);
                    double* al = a + l * N;
                    cheb_scaled(zeta, N, al);
                    for (int k = 0; k < N; ++k) al[k] *= m2;
                }
                if (n_k > 0) {
                    for (int r = 0; r < n_k; ++r) {
                        double b = wt;
                        for (int l = 0; l < dim; ++l) b *= a[l * N + kidx[r * dim + l]];
                        sum2_add(&acc[r], &cmp[r], b);
                    }
                } else if (dim == 2) {
                    for (int k1 = 0; k1 < N; ++k1) {
                        double b1 = wt * a[k1];
                        double* row = acc + (size_t)k1 * N;
                        double* rowc = cmp + (size_t)k1 * N;
                        for (int k2 = 0; k2 < N; ++k2) sum2_add(&row[k2], &rowc[k2], b1 * a[N + k2]);
                    }
                } else {
                    for (int k1 = 0; k1 < N; ++k1) {
                        double b1 = wt * a[k1];
                        for (int k2 = 0; k2 < N; ++k2) {
                            double b2 = b1 * a[N + k2];
                            double* row = acc + ((size_t)k1 * N + k2) * N;
                            double* rowc = cmp + ((size_t)k1 * N + k2) * N;
                            for (int k3 = 0; k3 < N; ++k3)
                                sum2_add(&row[k3], &rowc[k3], b2 * a[2 * N + k3]);
                        }
                    }
                }
            }
        }
        free(a);
    }
    for (int64_t k = 0; k < nout; ++k) {
        double s = 0.0, c = 0.0;
        for (int th = 0; th < nth; ++th) {
            sum2_add(&s, &c, part[(size_t)th * 2 * nout + k]);
            c += part[(size_t)th * 2 * nout + nout + k];
        }
        out[k] = s + c;
    }
    free(part);
}

static void loss_sum(const ora_problem* p, const ora_tables* t, const ora_nodes* nd,
                     int n_k, const int* kidx, double* out)
{
    int dim = t->dim, N = t->N;
    double* A = (double*)malloc(sizeof(double) * t->nd);
    loss_field(p, t, nd, A);
    int64_t nout = n_k > 0 ? n_k : t->Nd;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nout; ++r) {
        int kk[3];
        if (n_k > 0) {
            for (int l = 0; l < dim; ++l) kk[l] = kidx[r * dim + l];
        } else {
            unflat(r, dim, N, kk);
        }
        double s = 0.0;
        for (int64_t i = 0; i < t->nd; ++i) {
            int ii[3];
            unflat(i, dim, t->ni, ii);
            double b = nd->w[i] * A[i] * nd->P[i];
            for (int l = 0; l < dim; ++l) b *= t->tn[(size_t)ii[l] * N + kk[l]];
            s += b;
        }
        out[r] = s;
    }
    free(A);
}

static int check_sphere(const ora_problem* p)
{
    if (p->n_sigma < 1 || !p->sigma || !p->sigma_w) return -1;
    return 0;
}

int ora_collision(const ora_problem* p, const double* coeffs, double* q, double* qplus,
                  double* qminus)
{
    if (check_problem(p) || check_sphere(p)) return -1;
    ora_tables t;
    tables_init(p, &t);
    ora_nodes nd;
    nodes_init(&t, coeffs, &nd);
    double* gp = (double*)malloc(sizeof(double) * t.Nd);
    double* gm = (double*)malloc(sizeof(double) * t.Nd);
    gain_sum(p, &t, &nd, 0, NULL, 0, (int64_t)p->n_sigma * t.nd, gp);
    loss_sum(p, &t, &nd, 0, NULL, gm);
    for (int64_t k = 0; k < t.Nd; ++k) {
        if (q) q[k] = gp[k] - gm[k];
        if (qplus) qplus[k] = gp[k];
        if (qminus) qminus[k] = gm[k];
    }
    free(gp);
    free(gm);
    nodes_free(&nd);
    tables_free(&t);
    return 0;
}

int ora_collision_at(const ora_problem* p, const double* coeffs, int n_k, const int* kidx,
                     double* qplus, double* qminus)
{
    if (check_problem(p) || check_sphere(p) || n_k < 1 || !kidx) return -1;
    for (int r = 0; r < n_k * p->dim; ++r)
        if (kidx[r] < 0 || kidx[r] >= p->n_modes) return -1;
    ora_tables t;
    tables_init(p, &t);
    ora_nodes nd;
    nodes_init(&t, coeffs, &nd);
    if (qplus) gain_sum(p, &t, &nd, n_k, kidx, 0, (int64_t)p->n_sigma * t.nd, qplus);
    if (qminus) loss_sum(p, &t, &nd, n_k, kidx, qminus);
    nodes_free(&nd);
    tables_free(&t);
    return 0;
}

int ora_gain_units(const ora_problem* p, const double* coeffs, int64_t u_lo, int64_t u_hi,
                   double* qplus)
{
    if (check_problem(p) || check_sphere(p)) return -1;
    ora_tables t;
    tables_init(p, &t);
    if (u_lo < 0 || u_hi < u_lo || u_hi > (int64_t)p->n_sigma * t.nd) {
        tables_free(&t);
        return -1;
    }
    ora_nodes nd;
    nodes_init(&t, coeffs, &nd);
    gain_sum(p, &t, &nd, 0, NULL, u_lo, u_hi, qplus);
    nodes_free(&nd);
    tables_free(&t);
    return 0;
}

int ora_eval(int dim, int n_modes, int map, double S, const double* coeffs, int64_t n,
             const double* v, double* out)
{
    if ((dim != 2 && dim != 3) || n_modes < 1 || S <= 0.0) return -1;
    int N = n_modes;
    int64_t Nd = ipow(N, dim);
#pragma omp parallel
    {
        double* a = (double*)malloc(sizeof(double) * 3 * N);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            for (int l = 0; l < dim; ++l) {
                double x = v[r * dim + l];
                double* al = a + l * N;
                cheb_scaled(map_xi(map, S, x), N, al);
                double m4 = mu4_of_v(map, S, x);
                for (int k = 0; k < N; ++k) al[k] *= m4;
            }
            double s = 0.0;
            for (int64_t k = 0; k < Nd; ++k) {
                int kk[3];
                unflat(k, dim, N, kk);
                double b = coeffs[k];
                for (int l = 0; l < dim; ++l) b *= a[l * N + kk[l]];
                s += b;
            }
            out[r] = s;
        }
        free(a);
    }
    return 0;
}

/* m_p[k] = int v^p T~_k(v) dv.
 * r = 1: closed forms from the substitution xi = cos(theta), as in the proof
 *        of the conservation theorem of Sec. 3.2:
 *          p = 0: (1/(S sqrt c_k)) int T_k sqrt(1 - xi^2) dxi,
 *          p = 1: (1/sqrt c_k) int xi T_k dxi,
 *          p = 2: (S/sqrt c_k) int xi^2 T_k (1 - xi^2)^{-1/2} dxi.
 * r = 0: trapezoid rule in v on [-80 S, 80 S], step S/64; the integrand
 *        v^p sech^2(v/S) T_k(tanh(v/S)) / (S^2 sqrt c_k) is analytic in a strip
 *        and decays like exp(-2|v|/S), so the rule converges geometrically. */
int ora_moment_functionals(int n_modes, int map, double S, int pmax, double* out)
{
    int N = n_modes;
    if (N < 1 || S <= 0.0 || pmax < 0) return -1;
    if (map == 1) {
        if (pmax > 2) return -1;
        for (int k = 0; k < N; ++k) {
            double sc = sqrt(cheb_norm(k));
            /* int_0^pi cos(k t) sin^2 t dt */
            double i0 = (k == 0) ? ORA_PI / 2 : (k == 2 ? -ORA_PI / 4 : 0.0);
            out[k] = i0 / (S * sc);
            if (pmax >= 1) {
                /* int_{-1}^{1} xi T_k dxi, using xi T_k = (T_{k+1} + T_{k-1})/2 and
                 * int T_n = (1 + (-1)^n)/(1 - n^2) for n != 1, 0 for n = 1 */
                double i1;
                if (k == 0) i1 = 0.0;
                else {
                    double a = 0.0;
                    int n1 = k + 1, n2 = k - 1;
                    if (n1 != 1) a += (1.0 + ((n1 & 1) ? -1.0 : 1.0)) / (1.0 - (double)n1 * n1);
                    if (n2 != 1) a += (1.0 + ((n2 & 1) ? -1.0 : 1.0)) / (1.0 - (double)n2 * n2);
                    i1 = 0.5 * a;
                }
                out[N + k] = i1 / sc;
            }
            if (pmax >= 2) {
                /* int_0^pi cos^2 t cos(k t) dt */
                double i2 = (k == 0) ? ORA_PI / 2 : (k == 2 ? ORA_PI / 4 : 0.0);
                out[2 * N + k] = S * i2 / sc;
            }
        }
        return 0;
    }
    if (map != 0) return -1;
    double h = S / 64.0;
    int64_t M = (int64_t)(80.0 * S / h);
    double* tk = (double*)malloc(sizeof(double) * N);
    for (int pp = 0; pp <= pmax; ++pp)
        for (int k = 0; k < N; ++k) out[pp * N + k] = 0.0;
    for (int64_t r = -M; r <= M; ++r) {
        double v = r * h;
        double c = cosh(v / S);
        double wgt = h / (c * c * S * S);
        cheb_scaled(tanh(v / S), N, tk);
        double vp = 1.0;
        for (int pp = 0; pp <= pmax; ++pp) {
            for (int k = 0; k < N; ++k) out[pp * N + k] += wgt * vp * tk[k];
            vp *= v;
        }
    }
    free(tk);
    return 0;
}

/* rho, rho u_l and E of f_N, the quantities of eq. (def_mom) */
int ora_moments(int dim, int n_modes, int map, double S, const double* coeffs, double* out)
{
    if (dim != 2 && dim != 3) return -1;
    int N = n_modes;
    double* m = (double*)malloc(sizeof(double) * 3 * N);
    if (ora_moment_functionals(N, map, S, 2, m)) {
        free(m);
        return -1;
    }
    int64_t Nd = ipow(N, dim);
    double res[5] = {0, 0, 0, 0, 0};
    for (int64_t k = 0; k < Nd; ++k) {
        int kk[3];
        unflat(k, dim, N, kk);
        double c = coeffs[k];
        double m0 = c;
        for (int l = 0; l < dim; ++l) m0 *= m[kk[l]];
        res[0] += m0;
        for (int l = 0; l < dim; ++l) {
            double a = c, e = c;
            for (int l2 = 0; l2 < dim; ++l2) {
                a *= (l2 == l) ? m[N + kk[l2]] : m[kk[l2]];
                e *= (l2 == l) ? m[2 * N + kk[l2]] : m[kk[l2]];
            }
            res[1 + l] += a;
            res[1 + dim] += e;
        }
    }
    for (int r = 0; r < dim + 2; ++r) out[r] = res[r];
    free(m);
    return 0;
}

/* classical fourth-order Runge-Kutta on the ODE system (spectral_ODE) */
int ora_rk4(const ora_problem* p, double* coeffs, double dt, int n_steps)
{
    if (check_problem(p) || check_sphere(p) || n_steps < 0) return -1;
    int64_t Nd = ipow(p->n_modes, p->dim);
    double* k1 = (double*)malloc(sizeof(double) * Nd);
    double* k2 = (double*)malloc(sizeof(double) * Nd);
    double* k3 = (double*)malloc(sizeof(double) * Nd);
    double* k4 = (double*)malloc(sizeof(double) * Nd);
    double* y = (double*)malloc(sizeof(double) * Nd);
    for (int st = 0; st < n_steps; ++st) {
        ora_collision(p, coeffs, k1, NULL, NULL);
        for (int64_t k = 0; k < Nd; ++k) y[k] = coeffs[k] + 0.5 * dt * k1[k];
        ora_collision(p, y, k2, NULL, NULL);
        for (int64_t k = 0; k < Nd; ++k) y[k] = coeffs[k] + 0.5 * dt * k2[k];
        ora_collision(p, y, k3, NULL, NULL);
        for (int64_t k = 0; k < Nd; ++k) y[k] = coeffs[k] + dt * k3[k];
        ora_collision(p, y, k4, NULL, NULL);
        for (int64_t k = 0; k < Nd; ++k)
            coeffs[k] += dt / 6.0 * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
    }
    free(k1);
    free(k2);
    free(k3);
    free(k4);
    free(y);
    return 0;
}

int ora_cosine_sum(int dim, int64_t n_pts, const double* z, const double* q, int n_modes,
                   double* out)
{
    if ((dim < 1 || dim > 3) || n_modes < 1 || n_pts < 0) return -1;
    int N = n_modes;
    int64_t Nd = ipow(N, dim);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < Nd; ++k) {
        int kk[3];
        unflat(k, dim, N, kk);
        double s = 0.0;
        for (int64_t r = 0; r < n_pts; ++r) {
            double b = q[r];
            for (int l = 0; l < dim; ++l) b *= cos(kk[l] * z[r * dim + l]);
            s += b;
        }
        out[k] = s;
    }
    return 0;
}
