/*
 * pgc_oracle.h -- plain FP64 CPU oracle for the Petrov-Galerkin mapped-Chebyshev
 * collision coefficients of Hu, Huang, Shen and Yang (arXiv 2105.08806).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * It shares no code with it.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load it; the product path never does.
 *
 * Conventions (all arrays host memory, row-major, last index fastest):
 *   N      modes per dimension, k = 0..N-1 (the paper's degree N-1).
 *   m_v    Chebyshev-Gauss-Lobatto nodes per dimension, both endpoints
 *          included; the n_i = m_v - 2 interior nodes carry every sum.
 *   map    0 = logarithmic map (r = 0), 1 = algebraic map (r = 1)  (Sec. 2.1).
 *   kernel 0 = Maxwell molecules, B = b0;
 *          1 = variable hard spheres, B = b0 |v - v_*|^gamma.
 * Every function returns 0 on success and a negative value on bad arguments.
 */
#ifndef PGC_ORACLE_H
#define PGC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int dim;               /* 2 or 3 */
    int n_modes;           /* N */
    int m_v;               /* CGL nodes per dimension incl. endpoints */
    int map;               /* 0: r = 0, 1: r = 1 */
    double S;              /* map scale */
    int kernel;            /* 0 Maxwell, 1 VHS, 2 angle-dependent */
    double b0;             /* kernel constant */
    double gamma;          /* exponent of |u| (kernels 1 and 2) */
    int n_sigma;           /* quadrature points on the unit sphere / circle */
    const double* sigma;   /* n_sigma x dim unit vectors */
    const double* sigma_w; /* n_sigma weights */
    double aniso;          /* kernel 2: B = b0 |u|^gamma (1 + aniso cos^2 theta), aniso >= -1 */
} ora_problem;

/* CGL nodes xi_j = -cos(pi j/(m_v-1)), weights, mapped v_j and mu(xi_j)^2
 * for j = 0..m_v-1 (endpoints: v = -/+HUGE_VAL, mu^2 = 0). */
int ora_cgl(int m_v, int map, double S, double* xi, double* v, double* w, double* mu2);

/* Circle rule theta_s = 2 pi s / m, W_s = 2 pi / m. */
int ora_circle_rule(int m, double* sigma, double* w);
/* Product sphere rule: n_t Gauss-Legendre nodes in cos(theta) x n_p uniform phi. */
int ora_sphere_product_rule(int n_t, int n_p, double* sigma, double* w);
/* Gauss-Legendre nodes/weights on [-1, 1]. */
int ora_gauss_legendre(int n, double* x, double* w);

/* f_k = sum over interior nodes of w_i mu_i^-4 f(v_i) T_k(xi_i)/sqrt(c_k).
 * f_int: n_i^dim values at the interior nodes; coeffs: N^dim. */
int ora_project(const ora_problem* p, const double* f_int, double* coeffs);
/* Polynomial part P_i = sum_k f_k T_k(xi_i)/sqrt(c_k) at the interior nodes. */
int ora_nodal(const ora_problem* p, const double* coeffs, double* P_int);

/* The discrete collision coefficients Q_k = Q+_k - Q-_k (N^dim each).  Any
 * output pointer may be NULL. */
int ora_collision(const ora_problem* p, const double* coeffs,
                  double* q, double* qplus, double* qminus);
/* The same sums for n_k selected multi-indices kidx (n_k x dim) only. */
int ora_collision_at(const ora_problem* p, const double* coeffs, int n_k,
                     const int* kidx, double* qplus, double* qminus);
/* The gain restricted to the collision units u = s * n_i^dim + i with
 * u_lo <= u < u_hi (all N^dim outputs); the units partition the sum. */
int ora_gain_units(const ora_problem* p, const double* coeffs, int64_t u_lo, int64_t u_hi,
                   double* qplus);

/* sum_k c_k T~_k(v) at n velocities v (n x dim). */
int ora_eval(int dim, int n_modes, int map, double S, const double* coeffs,
             int64_t n, const double* v, double* out);

/* 1D moment functionals m_p[k] = int v^p T~_k(v) dv, p = 0..pmax, out is
 * (pmax+1) x N.  For map = 1 only pmax <= 2 exists. */
int ora_moment_functionals(int n_modes, int map, double S, int pmax, double* out);
/* Mass, momentum (dim values) and energy int |v|^2 f of sum_k c_k T~_k. */
int ora_moments(int dim, int n_modes, int map, double S, const double* coeffs, double* out);

/* Classical RK4 on d f_k/dt = Q_k, n_steps steps of size dt, in place. */
int ora_rk4(const ora_problem* p, double* coeffs, double dt, int n_steps);

/* Direct cosine sum out_k = sum_p q_p prod_l cos(k_l z_{p,l}), k < n_modes. */
int ora_cosine_sum(int dim, int64_t n_pts, const double* z, const double* q,
                   int n_modes, double* out);

int ora_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
