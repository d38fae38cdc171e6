/*
 * pf_oracle.c -- plain, slow, FP64 CPU oracle for the explicit phase-field +
 * concentration time step of Seiz & Takaki, "Numerical efficiency of explicit
 * time integrators for phase-field models" (arXiv 2601.16522).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * implementation.
 *
 * Everything is IEEE double, evaluated left to right as written (compile with
 * -ffp-contract=off so no fused multiply-add is formed).  Each routine names
 * the passage of the paper it follows.  Where the paper is silent or garbled
 * the reading taken is named "reading Rn" (the list of readings is kept with
 * the design notes of the repository).
 *
 * State vector layout: F = n_phi + with_c planes of V = nx*ny*nz doubles,
 * plane a < n_phi holds phi_a, plane n_phi holds c; x runs fastest, then y,
 * then z.  Boundaries are periodic unless stated (Sec. 4, "Common
 * conditions"); an axis may instead end in walls where phi and c have zero
 * gradient, and a wall face may hold c at a fixed value (the Dirichlet
 * condition of the solutal Stefan problem, Sec. 5.2.2; reading in the
 * design notes: the ghost cell beyond the face takes the wall cell's phi and
 * the fixed c).
 *
 * Parity status of each part (how each is pinned is in tests/):
 *   variational derivative, RHS, simplex, integrators, stable step, estimator:
 *     pinned (energy brute force, closed forms, Legendre stability
 *     polynomials, Table 3, Taylor order).
 *   walls and fixed-c faces: pinned (the solutal Stefan growth constant of
 *     Sec. 5.2.2; plain diffusion against a fixed-c wall, erf solution).
 *   c coupling at equilibrium: pinned (phase embedding, Laplace pressure).
 *   RKL2 first-stage correction: pinned on clipped cells and by its effect
 *     on the error (Sec. 3.2 end).
 *   SSP(10)4 embedded solution: pinned by the order conditions of its
 *     Butcher tableau and its stability polynomial.
 *   PID controller: the printed gains recovered from its output through the
 *     inverted limiter, the reject fallback, bias and limiter invariants.
 *   error norm: pinned where every entry counts (the textbook weighted RMS
 *     norm) and, for the degree-of-freedom rule, by the paper's reason for it
 *     (two phases held in more slots give the norm of a direct two-phase
 *     implementation); the phi filter of the estimate by hand-worked cases
 *     (the paper prints no worked example of it) that fail for a full dt in
 *     the trial value, an open interval, a filtered c entry, a trial without
 *     rhs(u^{n+1}) and a trial based on u^{n+1}.
 *   sparse storage rule: hand-worked cells; equal to dense storage bit for
 *     bit while nothing is cut.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PFO_MAXN 32
#define PFO_MAXT 4
#define PFO_PI 3.14159265358979323846

enum { PFO_FE = 0, PFO_SSP2 = 1, PFO_SSP104 = 2, PFO_RKL1 = 3, PFO_RKL2 = 4 };

typedef struct {
    int dim, nx, ny, nz;
    int n_phi, with_c, n_types;
    int type_of[PFO_MAXN];
    double dx, W;
    double gamma[PFO_MAXT * PFO_MAXT]; /* symmetric pair table over types */
    double mob[PFO_MAXT * PFO_MAXT];   /* symmetric pair table over types */
    double k[PFO_MAXT], c0[PFO_MAXT], D[PFO_MAXT];
    /* boundaries: bc[axis] 0 periodic, 1 walls (zero gradient); per face
     * (x-, x+, y-, y+, z-, z+) of a walled axis, c_fixed[face] != 0 holds c
     * at c_bc[face] in the ghost cell */
    int bc[3];
    int c_fixed[6];
    double c_bc[6];
    /* sparse phase storage (Sec. 3.1 "Phase-field details"; reading R23):
     * n_p > 0 keeps at most n_p nonzero phi per cell, see cell_store; 0 keeps
     * all N (dense) */
    int n_p;
} pfo_params;

typedef struct {
    double r_phi, a_phi, r_c, a_c;
    double dt_max_over_dte;
    double dt0;
} pfo_tol;

typedef struct {
    long long rhs_evals, stages, accepted, rejected;
    double t, last_dt, last_err;
} pfo_stats;

static long long ncells(const pfo_params *P) { return (long long)P->nx * P->ny * P->nz; }
static int nfields(const pfo_params *P) { return P->n_phi + (P->with_c ? 1 : 0); }

/* ---------------------------------------------------------------------------
 * Model constants (Sec. 2, below eq. profile): for the pair (a,b) with types
 * (ta,tb):  A = 4 W gamma / pi,  B = 4 gamma / (pi W),  L = pi M / (4 W).
 * ------------------------------------------------------------------------- */
static double pair_A(const pfo_params *P, int a, int b) {
    double g = P->gamma[P->type_of[a] * P->n_types + P->type_of[b]];
    return 4.0 * P->W * g / PFO_PI;
}
static double pair_B(const pfo_params *P, int a, int b) {
    double g = P->gamma[P->type_of[a] * P->n_types + P->type_of[b]];
    return 4.0 * g / (PFO_PI * P->W);
}
static double pair_L(const pfo_params *P, int a, int b) {
    double m = P->mob[P->type_of[a] * P->n_types + P->type_of[b]];
    return PFO_PI * m / (4.0 * P->W);
}

void pfo_pair_constants(const pfo_params *P, double *A, double *B, double *L) {
    int N = P->n_phi;
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            A[a * N + b] = pair_A(P, a, b);
            B[a * N + b] = pair_B(P, a, b);
            L[a * N + b] = pair_L(P, a, b);
        }
}

/* Neighbour coordinate of q in direction s (-1 or +1) on an axis of n cells:
 * wrapped when periodic; at a wall the cell itself (zero gradient), and
 * *ghost = 1. */
static long long nb_coord(long long q, int s, long long n, int walls, int *ghost) {
    long long r = q + s;
    *ghost = 0;
    if (r >= 0 && r < n) return r;
    if (!walls) return (r + n) % n;
    *ghost = 1;
    return q;
}

/* Neighbour list of cell i: x-, x+, y-, y+, (z-, z+).  ghost[k] is the face
 * index k when neighbour k lies beyond a wall (then nb[k] = i), else -1. */
static int neighbours_g(const pfo_params *P, long long i, long long *nb, int *ghost) {
    long long nx = P->nx, ny = P->ny, nz = P->nz;
    long long x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    int g;
    int nnb = P->dim == 3 ? 6 : 4;
    for (int k = 0; k < nnb; ++k) {
        const int axis = k / 2, s = (k & 1) ? 1 : -1;
        long long xx = x, yy = y, zz = z;
        if (axis == 0) xx = nb_coord(x, s, nx, P->bc[0], &g);
        else if (axis == 1) yy = nb_coord(y, s, ny, P->bc[1], &g);
        else zz = nb_coord(z, s, nz, P->bc[2], &g);
        nb[k] = (zz * ny + yy) * nx + xx;
        ghost[k] = g ? k : -1;
    }
    return nnb;
}

static int neighbours(const pfo_params *P, long long i, long long *nb) {
    int ghost[6];
    return neighbours_g(P, i, nb, ghost);
}

/* ---------------------------------------------------------------------------
 * KKS chemical potential with parabolic g (eqs. cadef, mueq, gibbs-energy):
 * c_a = c0_a + mu/k_a and c = sum_a phi_a c_a give
 *     mu = (c - sum_a phi_a c0_a) / (sum_a phi_a / k_a).
 * The division by k is taken as a product with 1/k, formed once per type.
 * Diffusive mobility (eq. ceq):  Mc = sum_a D_a phi_a / k_a.
 * ------------------------------------------------------------------------- */
static void cell_mu_mc(const pfo_params *P, const double *u, long long V, long long i,
                       double *mu, double *mc) {
    int N = P->n_phi;
    double sc0 = 0.0, sik = 0.0, smc = 0.0;
    for (int a = 0; a < N; ++a) {
        int t = P->type_of[a];
        double ik = 1.0 / P->k[t];
        double p = u[(long long)a * V + i];
        sc0 = sc0 + p * P->c0[t];
        sik = sik + p * ik;
        smc = smc + p * (P->D[t] * ik);
    }
    *mu = (u[(long long)N * V + i] - sc0) / sik;
    *mc = smc;
}

/* mu of a ghost cell beyond a face that holds c at cf: the wall cell's phi
 * with c = cf (the same formula as cell_mu_mc). */
static double ghost_mu(const pfo_params *P, const double *u, long long V, long long i, double cf) {
    int N = P->n_phi;
    double sc0 = 0.0, sik = 0.0;
    for (int a = 0; a < N; ++a) {
        int t = P->type_of[a];
        double ik = 1.0 / P->k[t];
        double p = u[(long long)a * V + i];
        sc0 = sc0 + p * P->c0[t];
        sik = sik + p * ik;
    }
    return (cf - sc0) / sik;
}

void pfo_mu(const pfo_params *P, const double *u, double *mu, double *mc) {
    long long V = ncells(P);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < V; ++i) cell_mu_mc(P, u, V, i, &mu[i], &mc[i]);
}

/* Grand potential of type t (Sec. 2, last equation):
 * psi = -mu^2/(2k) - mu c0. */
static double grand_potential(const pfo_params *P, int t, double mu) {
    return -mu * mu / (2.0 * P->k[t]) - mu * P->c0[t];
}

/* Second-order five/seven-point Laplacian as a sum of face differences
 * (Sec. 3, "Spatial discretization"): (sum_nb u_nb - 2d u_i) / dx^2. */
static double laplacian(const pfo_params *P, const double *plane, long long i,
                        const long long *nb, int nnb) {
    double s = 0.0;
    for (int k = 0; k < nnb; ++k) s = s + plane[nb[k]];
    s = s - (double)nnb * plane[i];
    return s * (1.0 / (P->dx * P->dx));
}

/* ---------------------------------------------------------------------------
 * Variational derivative of F (eqs. energy, wterm, phieq second line) at every
 * cell and phase:
 *   delta_a = sum_{b != a} ( A_ab Lap phi_b + B_ab phi_b ) + psi_{t(a)}(mu)
 * since -div(d a / d grad phi_a) = + sum_b A_ab Lap phi_b and
 * d w / d phi_a = sum_b B_ab phi_b; d f / d phi_a at fixed c is psi_a (KKS).
 * Without c there is no chemical term.
 * ------------------------------------------------------------------------- */
static void cell_delta(const pfo_params *P, const double *u, long long V, long long i,
                       const double *mu, double *lap, double *delta) {
    int N = P->n_phi;
    long long nb[6];
    int nnb = neighbours(P, i, nb);
    for (int b = 0; b < N; ++b) lap[b] = laplacian(P, u + (long long)b * V, i, nb, nnb);
    for (int a = 0; a < N; ++a) {
        double s = 0.0;
        for (int b = 0; b < N; ++b) {
            if (b == a) continue;
            s = s + (pair_A(P, a, b) * lap[b] + pair_B(P, a, b) * u[(long long)b * V + i]);
        }
        if (P->with_c) s = s + grand_potential(P, P->type_of[a], mu[i]);
        delta[a] = s;
    }
}

void pfo_delta(const pfo_params *P, const double *u, double *delta_out) {
    long long V = ncells(P);
    int N = P->n_phi;
    double *mu = (double *)calloc((size_t)V, sizeof(double));
    double *mc = (double *)calloc((size_t)V, sizeof(double));
    if (P->with_c) pfo_mu(P, u, mu, mc);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < V; ++i) {
        double lap[PFO_MAXN], d[PFO_MAXN];
        cell_delta(P, u, V, i, mu, lap, d);
        for (int a = 0; a < N; ++a) delta_out[(long long)a * V + i] = d[a];
    }
    free(mu);
    free(mc);
}

/* ---------------------------------------------------------------------------
 * Right-hand side (eq. phieq with sign reading R2, eq. ceq with face
 * mobility reading R5/R6).
 *
 * Activity (reading R1 of the filter n and of N_z): phase a is active at cell
 * i when phi_a > 0 at i or at any of its 2d neighbours; N_z counts them.
 *   rphi_a = -(1/N_z) sum_{b active, b != a} L_ab (delta_a - delta_b)
 * for active a when N_z >= 2, otherwise 0.
 *   rc_i = (1/dx^2) sum_nb w_ij (mu_j - mu_i),  w_ij = (Mc_i + Mc_j)/2.
 * ------------------------------------------------------------------------- */
static void cell_rhs(const pfo_params *P, const double *u, long long V, long long i,
                     const double *mu, const double *mc, double *ri /* F values */) {
    int N = P->n_phi;
    long long nb[6];
    int ghost[6];
    int nnb = neighbours_g(P, i, nb, ghost);
    int act[PFO_MAXN];
    int nz = 0;
    for (int a = 0; a < N; ++a) {
        const double *pa = u + (long long)a * V;
        int on = pa[i] > 0.0;
        for (int k = 0; k < nnb; ++k) on = on || (pa[nb[k]] > 0.0);
        act[a] = on;
        nz += on;
    }
    double lap[PFO_MAXN], delta[PFO_MAXN];
    cell_delta(P, u, V, i, mu, lap, delta);
    for (int a = 0; a < N; ++a) {
        double ra = 0.0;
        if (act[a] && nz >= 2) {
            double s = 0.0;
            for (int b = 0; b < N; ++b) {
                if (b == a || !act[b]) continue;
                s = s + pair_L(P, a, b) * (delta[a] - delta[b]);
            }
            ra = -s * (1.0 / (double)nz);
        }
        ri[a] = ra;
    }
    if (P->with_c) {
        double s = 0.0;
        for (int k = 0; k < nnb; ++k) {
            double w = 0.5 * (mc[i] + mc[nb[k]]);
            double muk = mu[nb[k]];
            /* a ghost cell that holds c fixed: the wall cell's phi (so the
             * same Mc) with the fixed c */
            if (ghost[k] >= 0 && P->c_fixed[ghost[k]]) muk = ghost_mu(P, u, V, i, P->c_bc[ghost[k]]);
            s = s + w * (muk - mu[i]);
        }
        ri[N] = s * (1.0 / (P->dx * P->dx));
    }
}

void pfo_rhs(const pfo_params *P, const double *u, double *r) {
    long long V = ncells(P);
    int N = P->n_phi;
    double *mu = (double *)calloc((size_t)V, sizeof(double));
    double *mc = (double *)calloc((size_t)V, sizeof(double));
    if (P->with_c) pfo_mu(P, u, mu, mc);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < V; ++i) {
        double ri[PFO_MAXN + 1];
        cell_rhs(P, u, V, i, mu, mc, ri);
        for (int a = 0; a < N; ++a) r[(long long)a * V + i] = ri[a];
        if (P->with_c) r[(long long)N * V + i] = ri[N];
    }
    free(mu);
    free(mc);
}

/* The right-hand side at n listed cells only (the same per-cell formula as
 * pfo_rhs; mu and Mc are formed over the whole grid): out[k * F + f] is field
 * f at cell cells[k].  For checking a large grid at sampled cells. */
void pfo_rhs_at(const pfo_params *P, const double *u, const long long *cells, long long n,
                double *out) {
    long long V = ncells(P);
    int F = P->n_phi + (P->with_c ? 1 : 0);
    double *mu = (double *)calloc((size_t)V, sizeof(double));
    double *mc = (double *)calloc((size_t)V, sizeof(double));
    if (P->with_c) pfo_mu(P, u, mu, mc);
#pragma omp parallel for schedule(static)
    for (long long k = 0; k < n; ++k) {
        double ri[PFO_MAXN + 1];
        cell_rhs(P, u, V, cells[k], mu, mc, ri);
        for (int f = 0; f < F; ++f) out[k * F + f] = ri[f];
    }
    free(mu);
    free(mc);
}

/* ---------------------------------------------------------------------------
 * Simplex projection S (Sec. 3.1, last paragraph; reading R19 for ties):
 * negatives become 0; if some phi_a >= 1 the largest of them (lowest index on
 * ties) becomes 1 and all others 0; finally divide by the sum.  A zero sum
 * (impossible from a state on the simplex) leaves the cell as clamped.
 * Returns the number of cells whose phi changed in any bit.
 * ------------------------------------------------------------------------- */
static int cell_simplex(int N, double *p /* N values */) {
    double old[PFO_MAXN];
    for (int a = 0; a < N; ++a) old[a] = p[a];
    for (int a = 0; a < N; ++a)
        if (p[a] < 0.0) p[a] = 0.0;
    int m = -1;
    for (int a = 0; a < N; ++a)
        if (p[a] >= 1.0 && (m < 0 || p[a] > p[m])) m = a;
    if (m >= 0)
        for (int a = 0; a < N; ++a) p[a] = (a == m) ? 1.0 : 0.0;
    double s = 0.0;
    for (int a = 0; a < N; ++a) s = s + p[a];
    if (s > 0.0)
        for (int a = 0; a < N; ++a) p[a] = p[a] / s;
    int changed = 0;
    for (int a = 0; a < N; ++a) changed |= memcmp(&old[a], &p[a], sizeof(double)) != 0;
    return changed;
}

/* Sparse phase storage (Sec. 3.1, "Phase-field details"): a cell holds at
 * most n_p phase values and their phase ids, the others being zero.  Reading
 * R23 for a cell with more than n_p nonzero phi: the n_p largest are kept
 * (equal values: the lower phase index first), the others become 0, and the
 * kept ones are divided by their sum, as the last step of S does.  A cell with
 * at most n_p nonzero values is left exactly as it is, so with n_p at least
 * the largest local phase count sparse storage gives the dense results.
 * Returns 1 when the cell changed. */
static long long store_truncations = 0; /* cells changed by the rule since the last reset */

static int cell_store(int N, int n_p, double *p) {
    int cnt = 0;
    for (int a = 0; a < N; ++a) cnt += p[a] != 0.0;
    if (n_p <= 0 || cnt <= n_p) return 0;
#pragma omp atomic
    store_truncations++;
    int keep[PFO_MAXN] = {0};
    for (int k = 0; k < n_p; ++k) {
        int m = -1;
        for (int a = 0; a < N; ++a)
            if (!keep[a] && p[a] != 0.0 && (m < 0 || p[a] > p[m])) m = a;
        keep[m] = 1;
    }
    double s = 0.0;
    for (int a = 0; a < N; ++a) {
        if (!keep[a]) p[a] = 0.0;
        s = s + p[a];
    }
    if (s > 0.0)
        for (int a = 0; a < N; ++a) p[a] = p[a] / s;
    return 1;
}

/* Number of cells the storage rule changed since the last call (the call
 * resets it): tells whether a sparse run ever dropped a phase. */
long long pfo_store_truncations(void) {
    long long n = store_truncations;
    store_truncations = 0;
    return n;
}

/* The storage rule alone on every cell (an initial state in sparse storage). */
long long pfo_store(const pfo_params *P, double *u) {
    long long V = ncells(P);
    int N = P->n_phi;
    long long n = 0;
    if (P->n_p <= 0) return 0;
#pragma omp parallel for schedule(static) reduction(+ : n)
    for (long long i = 0; i < V; ++i) {
        double p[PFO_MAXN];
        for (int a = 0; a < N; ++a) p[a] = u[(long long)a * V + i];
        int ch = cell_store(N, P->n_p, p);
        for (int a = 0; a < N; ++a) u[(long long)a * V + i] = p[a];
        n += ch;
    }
    return n;
}

/* S followed by the storage rule (every stored stage of a sparse run). */
long long pfo_simplex(const pfo_params *P, double *u, unsigned char *changed_out) {
    long long V = ncells(P);
    int N = P->n_phi;
    long long nchanged = 0;
#pragma omp parallel for schedule(static) reduction(+ : nchanged)
    for (long long i = 0; i < V; ++i) {
        double p[PFO_MAXN];
        for (int a = 0; a < N; ++a) p[a] = u[(long long)a * V + i];
        int ch = cell_simplex(N, p);
        ch |= cell_store(N, P->n_p, p);
        for (int a = 0; a < N; ++a) u[(long long)a * V + i] = p[a];
        if (changed_out) changed_out[i] = (unsigned char)ch;
        nchanged += ch;
    }
    return nchanged;
}

/* ---------------------------------------------------------------------------
 * Runge-Kutta-Legendre coefficients (Meyer et al. 2012, 2014; the recursion
 * is eq. sts).  Index j = 1..s.  For RKL1:
 *   w1 = 2/(s^2+s), mut_1 = w1, mu_j = (2j-1)/j, nu_j = (1-j)/j,
 *   mut_j = w1 mu_j, gam_j = 0.
 * For RKL2 (s >= 2), with b_0 = b_1 = b_2 = 1/3, b_j = (j^2+j-2)/(2j(j+1)),
 * a_j = 1 - b_j:
 *   w1 = 4/(s^2+s-2), mut_1 = b_1 w1,
 *   mu_j = (2j-1)/j * b_j/b_{j-1}, nu_j = -(j-1)/j * b_j/b_{j-2},
 *   mut_j = mu_j w1, gam_j = -a_{j-1} mut_j.
 * ------------------------------------------------------------------------- */
static double rkl2_b(int j) {
    if (j < 3) return 1.0 / 3.0;
    return ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
}

void pfo_rkl_coeffs(int order, int s, int j, double *mu, double *nu, double *mut, double *gam) {
    if (order == 1) {
        double w1 = 2.0 / ((double)s * s + s);
        if (j == 1) {
            *mu = 0.0; *nu = 0.0; *mut = w1; *gam = 0.0;
            return;
        }
        *mu = (2.0 * j - 1.0) / j;
        *nu = (1.0 - j) / j;
        *mut = w1 * *mu;
        *gam = 0.0;
        return;
    }
    double w1 = 4.0 / ((double)s * s + s - 2.0);
    if (j == 1) {
        *mu = 0.0; *nu = 0.0; *mut = rkl2_b(1) * w1; *gam = 0.0;
        return;
    }
    *mu = (2.0 * j - 1.0) / j * (rkl2_b(j) / rkl2_b(j - 1));
    *nu = -(j - 1.0) / j * (rkl2_b(j) / rkl2_b(j - 2));
    *mut = *mu * w1;
    *gam = -(1.0 - rkl2_b(j - 1)) * *mut;
}

/* ---------------------------------------------------------------------------
 * Integrators.  Every stage output has S applied to its phi planes
 * (Sec. 3.2: "the simplex constraint is applied to every stage").
 * ------------------------------------------------------------------------- */
static void project(const pfo_params *P, double *y) {
    pfo_simplex(P, y, NULL);
}

/* Forward Euler: u <- S(u + dt rhs(u)). */
static void step_fe(const pfo_params *P, double dt, double *u, double *r, pfo_stats *st) {
    long long n = (long long)nfields(P) * ncells(P);
    pfo_rhs(P, u, r);
    st->rhs_evals++; st->stages++;
    for (long long i = 0; i < n; ++i) u[i] = u[i] + dt * r[i];
    project(P, u);
}

/* SSP(s)2, Alg. ssp2 with the last line read as using the newest stage
 * (reading R7): s-1 projected Euler sub-steps q3 = S(q1 + dt (rhs(q1) / (s-1)))
 * in the algorithm's printed order (the RHS divided by s-1, then times dt),
 * then u^{n+1} = S(((s-1) q1 + u^n + dt rhs(q1)) / s).
 * z (optional) receives the last sub-step q1 = Y_{s-1}, the embedded
 * first-order solution of reading R9. */
static void step_ssp2(const pfo_params *P, int s, double dt, double *u, double *z,
                      double *r, double *q1, double *q3, pfo_stats *st) {
    long long n = (long long)nfields(P) * ncells(P);
    memcpy(q1, u, (size_t)n * sizeof(double));
    for (int i = 1; i <= s - 1; ++i) {
        pfo_rhs(P, q1, r);
        st->rhs_evals++; st->stages++;
        for (long long e = 0; e < n; ++e) q3[e] = q1[e] + dt * (r[e] / (s - 1));
        project(P, q3);
        double *tmp = q1; q1 = q3; q3 = tmp;
    }
    pfo_rhs(P, q1, r);
    st->rhs_evals++; st->stages++;
    for (long long e = 0; e < n; ++e) q3[e] = ((s - 1) * q1[e] + u[e] + dt * r[e]) / s;
    project(P, q3);
    if (z) memcpy(z, q1, (size_t)n * sizeof(double));
    memcpy(u, q3, (size_t)n * sizeof(double));
}

/* SSP(10)4, the low-storage ten-stage fourth-order scheme of Ketcheson (2008),
 * with S after every stage; the two linear combinations after the fifth stage
 * belong to that stage's output and the new q1 is projected.
 * z (optional) receives the tenth stage value Y_10 (q1 before the final
 * combination): as a Runge-Kutta solution its weights are 1/15 on the first
 * five stage RHS and 1/6 on the next four, which satisfy the conditions of
 * order 2 (sum b = 1, sum b c = 1/2) and not all of order 3 (sum b c^2 =
 * 11/36; on linear problems it is third order), so it is an embedded
 * lower-order solution that costs nothing (the embedded SSP estimate of
 * Sec. 3.3; reading R9). */
static void step_ssp104(const pfo_params *P, double dt, double *u, double *z, double *r,
                        double *q1, double *q2, double *q3, pfo_stats *st) {
    long long n = (long long)nfields(P) * ncells(P);
    memcpy(q1, u, (size_t)n * sizeof(double));
    memcpy(q2, u, (size_t)n * sizeof(double));
    for (int i = 1; i <= 9; ++i) {
        pfo_rhs(P, q1, r);
        st->rhs_evals++; st->stages++;
        for (long long e = 0; e < n; ++e) q3[e] = q1[e] + dt / 6.0 * r[e];
        project(P, q3);
        double *tmp = q1; q1 = q3; q3 = tmp;
        if (i == 5) {
            for (long long e = 0; e < n; ++e) q2[e] = 1.0 / 25.0 * q2[e] + 9.0 / 25.0 * q1[e];
            for (long long e = 0; e < n; ++e) q1[e] = 15.0 * q2[e] - 5.0 * q1[e];
            project(P, q1);
        }
    }
    pfo_rhs(P, q1, r);
    st->rhs_evals++; st->stages++;
    for (long long e = 0; e < n; ++e) u[e] = q2[e] + 3.0 / 5.0 * q1[e] + dt / 10.0 * r[e];
    project(P, u);
    if (z) memcpy(z, q1, (size_t)n * sizeof(double));
}

/* RKL1, Alg. sts1 with readings R10 (stage 1 uses mut_1; coefficients indexed
 * by the stage; S after stage 1 too), three-buffer ring. r0 (optional)
 * receives rhs(u^n) for the estimator. */
static void step_rkl1(const pfo_params *P, int s, double dt, double *u, double *r0,
                      double *r, double *q[3], pfo_stats *st) {
    long long n = (long long)nfields(P) * ncells(P);
    double mu, nu, mut, gam;
    memcpy(q[0], u, (size_t)n * sizeof(double));
    pfo_rhs(P, q[0], r);
    st->rhs_evals++; st->stages++;
    if (r0) memcpy(r0, r, (size_t)n * sizeof(double));
    pfo_rkl_coeffs(1, s, 1, &mu, &nu, &mut, &gam);
    for (long long e = 0; e < n; ++e) q[1][e] = q[0][e] + dt * mut * r[e];
    project(P, q[1]);
    int j = 1;
    for (int i = 2; i <= s; ++i) {
        j = i % 3;
        int jp = (i - 1) % 3, jpp = (i - 2) % 3;
        pfo_rhs(P, q[jp], r);
        st->rhs_evals++; st->stages++;
        pfo_rkl_coeffs(1, s, i, &mu, &nu, &mut, &gam);
        for (long long e = 0; e < n; ++e)
            q[j][e] = mu * q[jp][e] + nu * q[jpp][e] + dt * mut * r[e];
        project(P, q[j]);
    }
    memcpy(u, q[s % 3], (size_t)n * sizeof(double));
}

/* Whether step_rkl2 applies the first-stage correction of rhs(u^{n,0})
 * (Sec. 3.2, end).  Always on except where a test switches it off to measure
 * its effect on the error (the paper reports that it improves the error). */
static int rkl2_r0_correction = 1;
void pfo_set_rkl2_r0_correction(int on) { rkl2_r0_correction = on != 0; }

/* RKL2, eq. sts with the stored old solution u^{n,0} (kept in u, apart from
 * the three-slot ring of stages) and initial RHS, and the
 * first-stage correction of rhs(u^{n,0}) where S changed a cell (reading R13):
 *   R0_phi <- (S(u^{n,1}) - u^{n,0}) / (mut_1 dt)   on those cells only.
 * The corrected R0 is the rhs(u^n) of every later stage and of the error
 * estimate of Sec. 3.3 (reading R14). */
static void step_rkl2(const pfo_params *P, int s, double dt, double *u, double *r0_out,
                      double *r0, double *r, double *q[3], pfo_stats *st) {
    long long V = ncells(P);
    int N = P->n_phi;
    long long n = (long long)nfields(P) * V;
    double mu, nu, mut, gam;
    memcpy(q[0], u, (size_t)n * sizeof(double));
    pfo_rhs(P, q[0], r0);
    st->rhs_evals++; st->stages++;
    pfo_rkl_coeffs(2, s, 1, &mu, &nu, &mut, &gam);
    double mut1 = mut;
    for (long long e = 0; e < n; ++e) q[1][e] = q[0][e] + mut * dt * r0[e];
    unsigned char *changed = (unsigned char *)calloc((size_t)V, 1);
    pfo_simplex(P, q[1], changed);
    for (long long i = 0; i < V; ++i) {
        if (!changed[i] || !rkl2_r0_correction) continue;
        for (int a = 0; a < N; ++a) {
            long long e = (long long)a * V + i;
            r0[e] = (q[1][e] - u[e]) / (mut1 * dt);
        }
    }
    free(changed);
    for (int j = 2; j <= s; ++j) {
        int jc = j % 3, jp = (j - 1) % 3, jpp = (j - 2) % 3;
        pfo_rhs(P, q[jp], r);
        st->rhs_evals++; st->stages++;
        pfo_rkl_coeffs(2, s, j, &mu, &nu, &mut, &gam);
        for (long long e = 0; e < n; ++e)
            q[jc][e] = (1.0 - mu - nu) * u[e] + mu * q[jp][e] + nu * q[jpp][e] +
                       dt * (mut * r[e] + gam * r0[e]);
        project(P, q[jc]);
    }
    memcpy(u, q[s % 3], (size_t)n * sizeof(double));
    if (r0_out) memcpy(r0_out, r0, (size_t)n * sizeof(double));
}

/* One step of the chosen integrator at a fixed dt.  s is the stage count of
 * SSP(s)2 or of the RKL scheme.  aux (optional) receives rhs(u^n) (corrected
 * for RKL2) for RKL1/RKL2, or the embedded solution for SSP(s)2 and
 * SSP(10)4. */
int pfo_step(const pfo_params *P, int integ, int s, double dt, double *u, double *aux,
             pfo_stats *st) {
    long long n = (long long)nfields(P) * ncells(P);
    pfo_store(P, u);  /* a state held in sparse storage (no-op when dense) */
    double *w[5];
    for (int k = 0; k < 5; ++k) {
        w[k] = (double *)calloc((size_t)n, sizeof(double));
        if (!w[k]) return -2;
    }
    int rc = 0;
    switch (integ) {
    case PFO_FE: step_fe(P, dt, u, w[0], st); break;
    case PFO_SSP2:
        if (s < 2) { rc = -1; break; }
        step_ssp2(P, s, dt, u, aux, w[0], w[1], w[2], st);
        break;
    case PFO_SSP104: step_ssp104(P, dt, u, aux, w[0], w[1], w[2], w[3], st); break;
    case PFO_RKL1: {
        if (s < 1) { rc = -1; break; }
        double *q[3] = {w[1], w[2], w[3]};
        step_rkl1(P, s, dt, u, aux, w[0], q, st);
        break;
    }
    case PFO_RKL2: {
        if (s < 2) { rc = -1; break; }
        double *q[3] = {w[1], w[2], w[3]};
        step_rkl2(P, s, dt, u, aux, w[4], w[0], q, st);
        break;
    }
    default: rc = -1;
    }
    for (int k = 0; k < 5; ++k) free(w[k]);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Stable forward-Euler step (Sec. 3.2 "Gershgorin ... lambda_phi, lambda_c",
 * whose formulas are in the unavailable supplement; reading R12):
 *   lambda_phi = Mx gx (4d/dx^2 - 1/W^2)
 *                + [c coupled, dc0 != 0] (pi Mx / (8W)) kx (dc0^2 + |dc0|)
 *   lambda_c   = (4d Dx / dx^2) (1 + |dc0|/2)
 * x = maximum over type pairs / types, dc0 = max |c0_s - c0_t|;
 * dt_e = 2 / max(lambda_phi, lambda_c).
 * ------------------------------------------------------------------------- */
double pfo_stable_dt(const pfo_params *P) {
    int T = P->n_types, d = P->dim;
    double Mx = 0.0, gx = 0.0, kx = 0.0, Dx = 0.0, dc0 = 0.0;
    int used[PFO_MAXT] = {0};
    for (int a = 0; a < P->n_phi; ++a) used[P->type_of[a]] = 1;
    for (int s = 0; s < T; ++s) {
        if (!used[s]) continue;
        if (P->k[s] > kx) kx = P->k[s];
        if (P->D[s] > Dx) Dx = P->D[s];
        for (int t = 0; t < T; ++t) {
            if (!used[t]) continue;
            if (P->mob[s * T + t] > Mx) Mx = P->mob[s * T + t];
            if (P->gamma[s * T + t] > gx) gx = P->gamma[s * T + t];
            if (fabs(P->c0[s] - P->c0[t]) > dc0) dc0 = fabs(P->c0[s] - P->c0[t]);
        }
    }
    double idx2 = 1.0 / (P->dx * P->dx);
    double lphi = Mx * gx * (4.0 * d * idx2 - 1.0 / (P->W * P->W));
    double lam = lphi;
    if (P->with_c) {
        if (dc0 != 0.0) lam += (PFO_PI * Mx / (8.0 * P->W)) * kx * (dc0 * dc0 + dc0);
        double lc = 4.0 * d * Dx * idx2 * (1.0 + dc0 / 2.0);
        if (lc > lam) lam = lc;
    }
    return 2.0 / lam;
}

/* Stage count of an RKL step (eq. sts-limit, reading R11): the smallest odd s
 * (s >= 1 for RKL1, s >= 3 for RKL2) whose exact real stability bound
 *   RKL1: dt <= 0.9 dt_e (s^2+s)/2      RKL2: dt <= 0.9 dt_e (s^2+s-2)/4
 * holds.  Returns -1 for dt <= 0. */
int pfo_stage_count(int order, double dt, double dte) {
    if (!(dt > 0.0) || !(dte > 0.0)) return -1;
    double h = 0.9 * dte;
    int s = order == 1 ? 1 : 3;
    for (; s < 1000000; s += 2) {
        double lim = order == 1 ? h * ((double)s * s + s) / 2.0 : h * ((double)s * s + s - 2.0) / 4.0;
        if (dt <= lim) return s;
    }
    return -1;
}

/* ---------------------------------------------------------------------------
 * Local error estimates and weighted RMS norm (Sec. 3.3, eq. error_norm with
 * reading R16: weight r max(|u^n|,|u^{n+1}|) + a per field; N counts the phi
 * entries with nonzero e (a cell with none counts 2) plus one c entry per
 * cell).
 *
 * kind 0 (STS, Sommeijer; reading R14 for the sign):
 *   e_i = (12 (u^n_i - u^{n+1}_i) + 6 dt (R0_i + rhs(u^{n+1})_i)) / 15,
 *   and a phi entry whose trial value u^n + dt/2 (R0 + rhs(u^{n+1})) lies
 *   outside [0,1] has e_i = 0.
 * kind 1 (embedded, reading R9):  e_i = u^{n+1}_i - z_i.
 * aux = R0 for kind 0, z for kind 1.  Returns the norm, writes N.
 * ------------------------------------------------------------------------- */
double pfo_error_norm(const pfo_params *P, int kind, double dt, const double *un,
                      const double *unp1, const double *aux, const pfo_tol *tol,
                      long long *ndof_out, double *sumsq_out, pfo_stats *st) {
    long long V = ncells(P);
    int N = P->n_phi;
    long long n = (long long)nfields(P) * V;
    double *e = (double *)calloc((size_t)n, sizeof(double));
    if (kind == 0) {
        double *r1 = (double *)calloc((size_t)n, sizeof(double));
        pfo_rhs(P, unp1, r1);
        if (st) st->rhs_evals++;
        for (long long i = 0; i < n; ++i) {
            e[i] = (12.0 * (un[i] - unp1[i]) + 6.0 * dt * (aux[i] + r1[i])) / 15.0;
            if (i < (long long)N * V) {
                double trial = un[i] + dt / 2.0 * (aux[i] + r1[i]);
                if (trial < 0.0 || trial > 1.0) e[i] = 0.0;
            }
        }
        free(r1);
    } else {
        for (long long i = 0; i < n; ++i) e[i] = unp1[i] - aux[i];
    }
    double sum = 0.0;
    long long ndof = 0;
    for (long long i = 0; i < V; ++i) {
        int nt = 0;
        for (int a = 0; a < N; ++a) {
            long long k = (long long)a * V + i;
            if (e[k] != 0.0) {
                double w = tol->r_phi * fmax(fabs(un[k]), fabs(unp1[k])) + tol->a_phi;
                double q = e[k] / w;
                sum = sum + q * q;
                nt++;
            }
        }
        ndof += nt > 0 ? nt : 2;
        if (P->with_c) {
            long long k = (long long)N * V + i;
            double w = tol->r_c * fmax(fabs(un[k]), fabs(unp1[k])) + tol->a_c;
            double q = e[k] / w;
            sum = sum + q * q;
            ndof += 1;
        }
    }
    free(e);
    if (ndof_out) *ndof_out = ndof;
    if (sumsq_out) *sumsq_out = sum;
    return sqrt(sum / (double)ndof);
}

/* ---------------------------------------------------------------------------
 * PID step-size controller (Sec. 3.3, after eq. error_norm; reading R17):
 *   E_n = e_n / b
 *   F = (E_n^-k1 E_{n-1}^-k2 E_{n-2}^-k3)^(1/(P+1)) (dt_n/dt_{n-1})^k4 (dt_{n-1}/dt_{n-2})^k5
 *   dt_{n+1} = dt_n (1 + 5 atan((F-1)/5))
 * k = (1.25, 0.5, -0.6, 0.25, 0).  History holds accepted steps only; terms
 * without data are dropped.  On a rejection where F > 1, F = e_n^(-k1/(P+1)).
 * E values are floored at 1e-12; a non-finite e is a rejection with F = 0.
 * The bias is then updated: accept b <- min(sqrt(b), 0.98), reject
 * b <- max(b^2, 0.1).
 * ------------------------------------------------------------------------- */
typedef struct {
    double b;
    int nhist;          /* accepted steps recorded, capped at 2 */
    double E1, E2;      /* E of the last two accepted steps */
    double h1, h2;      /* their step sizes */
} pfo_ctrl;

void pfo_ctrl_init(pfo_ctrl *c) {
    c->b = 0.9; c->nhist = 0; c->E1 = c->E2 = 0.0; c->h1 = c->h2 = 0.0;
}

/* Returns the proposed next step; *accept is set from e < 1. */
double pfo_ctrl_update(pfo_ctrl *c, int order, double e, double h, int *accept) {
    const double k1 = 1.25, k2 = 0.5, k3 = -0.6, k4 = 0.25, k5 = 0.0;
    double p1 = order + 1.0;
    int finite = isfinite(e);
    int acc = finite && e < 1.0;
    double F;
    double E = e / c->b;
    if (E < 1e-12) E = 1e-12;
    if (!finite) {
        F = 0.0;
    } else {
        double prod = pow(E, -k1);
        if (c->nhist >= 1) prod = prod * pow(c->E1, -k2);
        if (c->nhist >= 2) prod = prod * pow(c->E2, -k3);
        F = pow(prod, 1.0 / p1);
        if (c->nhist >= 1) F = F * pow(h / c->h1, k4);
        if (c->nhist >= 2) F = F * pow(c->h1 / c->h2, k5);
        if (!acc && F > 1.0) {
            double en = e < 1e-12 ? 1e-12 : e;
            F = pow(en, -k1 / p1);
        }
    }
    double hn = h * (1.0 + 5.0 * atan((F - 1.0) / 5.0));
    if (acc) {
        c->E2 = c->E1; c->h2 = c->h1;
        c->E1 = E; c->h1 = h;
        if (c->nhist < 2) c->nhist++;
        double sb = sqrt(c->b);
        c->b = sb < 0.98 ? sb : 0.98;
    } else {
        double b2 = c->b * c->b;
        c->b = b2 > 0.1 ? b2 : 0.1;
    }
    *accept = acc;
    return hn;
}

static int method_order(int integ) {
    switch (integ) {
    case PFO_FE: return 1;
    case PFO_SSP2: return 2;
    case PFO_SSP104: return 4;
    case PFO_RKL1: return 1;
    default: return 2;
    }
}

/* ---------------------------------------------------------------------------
 * Integrate to t_end exactly (Sec. 5 opening, "output at defined target
 * times exactly"; reading R18): the step that would pass t_end is clipped to
 * land on it; an RKL stage count is recomputed for the clipped step.
 *
 * tol == NULL: fixed steps of dt_fixed (RKL stage count from dt and dt_e).
 * tol != NULL: adaptive RKL1/RKL2 (Sommeijer estimate) or SSP(s)2 and
 * SSP(10)4 (embedded estimate), PID controller, dt <= dt_max_over_dte * dt_e
 * (SSP(s)2 also <= 0.9 (s-1) dt_e, SSP(10)4 <= 0.9 * 6 dt_e: the schemes'
 * stability limits of Sec. 3.2 with the safety factor of the RKL stage
 * count), dt0 = tol->dt0 or 0.9 dt_e when that is <= 0.
 * trace (optional, 4 doubles per attempt: dt, s, e, accepted) records up to
 * trace_cap attempts.  ctrl_io/dt_io (optional): when *dt_io > 0 the adaptive
 * loop resumes that controller state and proposed step; both are written back.  Returns 0, or -5 when dt underflows, -4 after three
 * consecutive non-finite error norms (state = last accepted).
 * ------------------------------------------------------------------------- */
int pfo_run_to(const pfo_params *P, int integ, int s_ssp, double t0, double t_end,
               const pfo_tol *tol, double dt_fixed, double *u, pfo_stats *st,
               double *trace, long long trace_cap, long long *ntrace,
               pfo_ctrl *ctrl_io, double *dt_io) {
    long long n = (long long)nfields(P) * ncells(P);
    double dte = pfo_stable_dt(P);
    double t = t0;
    pfo_store(P, u);  /* a state held in sparse storage (no-op when dense) */
    long long nt = 0;
    if (ntrace) *ntrace = 0;
    if (!tol) {
        if (!(dt_fixed > 0.0)) return -1;
        for (;;) {
            double rem = t_end - t;
            /* a step of infinite size (reading R18 below) ends on t_end */
            if (rem <= 1e-12 * (isinf(dt_fixed) ? rem : dt_fixed)) break;
            double h = dt_fixed;
            int last = 0;
            if (rem <= h * (1.0 + 1e-10)) { h = rem; last = 1; }
            int s = s_ssp;
            if (integ == PFO_RKL1 || integ == PFO_RKL2)
                s = pfo_stage_count(integ == PFO_RKL1 ? 1 : 2, h, dte);
            int rc = pfo_step(P, integ, s, h, u, NULL, st);
            if (rc) return rc;
            st->accepted++;
            if (trace && nt < trace_cap) {
                trace[4 * nt] = h; trace[4 * nt + 1] = s; trace[4 * nt + 2] = 0.0; trace[4 * nt + 3] = 1.0;
            }
            nt++;
            t = last ? t_end : t + h;
            st->last_dt = h;
        }
        st->t = t;
        if (ntrace) *ntrace = nt;
        return 0;
    }
    if (integ != PFO_RKL1 && integ != PFO_RKL2 && integ != PFO_SSP2 && integ != PFO_SSP104)
        return -7;
    int order = method_order(integ);
    int embedded = integ == PFO_SSP2 || integ == PFO_SSP104;
    double dtmax = tol->dt_max_over_dte * dte;
    if (integ == PFO_SSP2) {
        double lim = 0.9 * (s_ssp - 1) * dte;
        if (lim < dtmax) dtmax = lim;
    }
    if (integ == PFO_SSP104) {
        double lim = 0.9 * 6.0 * dte;
        if (lim < dtmax) dtmax = lim;
    }
    double dt = tol->dt0 > 0.0 ? tol->dt0 : 0.9 * dte;
    double *y = (double *)calloc((size_t)n, sizeof(double));
    double *aux = (double *)calloc((size_t)n, sizeof(double));
    pfo_ctrl ctrl;
    pfo_ctrl_init(&ctrl);
    /* carry the controller over from a previous call (integration with output
     * times continues the same step-size sequence) */
    if (ctrl_io && dt_io && *dt_io > 0.0) {
        ctrl = *ctrl_io;
        if (!(tol->dt0 > 0.0)) dt = *dt_io;
    }
    int nonfinite = 0;
    int rc = 0;
    for (;;) {
        double rem = t_end - t;
        double h = dt < dtmax ? dt : dtmax;
        /* reading R18: the step that would pass t_end is clipped to the
         * remainder, an infinite one too (dt_e is infinite when no pair has
         * mobility and no phase diffuses: the right-hand side is zero); the
         * underflow test needs a finite dt_e */
        if (rem <= 1e-12 * (isinf(h) ? rem : h)) break;
        int last = 0;
        if (rem <= h * (1.0 + 1e-10)) { h = rem; last = 1; }
        if (!last && isfinite(dte) && h < 1e-12 * dte) { rc = -5; break; }
        int s = s_ssp;
        if (integ == PFO_SSP104) s = 10;
        else if (integ != PFO_SSP2) s = pfo_stage_count(order, h, dte);
        memcpy(y, u, (size_t)n * sizeof(double));
        rc = pfo_step(P, integ, s, h, y, aux, st);
        if (rc) break;
        double e = pfo_error_norm(P, embedded ? 1 : 0, h, u, y, aux, tol, NULL, NULL, st);
        int acc;
        double hn = pfo_ctrl_update(&ctrl, order, e, h, &acc);
        if (trace && nt < trace_cap) {
            trace[4 * nt] = h; trace[4 * nt + 1] = s; trace[4 * nt + 2] = e; trace[4 * nt + 3] = acc;
        }
        nt++;
        st->last_err = e;
        if (acc) {
            memcpy(u, y, (size_t)n * sizeof(double));
            t = last ? t_end : t + h;
            st->accepted++;
            st->last_dt = h;
            nonfinite = 0;
        } else {
            st->rejected++;
            if (!isfinite(e) && ++nonfinite >= 3) { rc = -4; break; }
        }
        dt = hn;
    }
    if (ctrl_io && dt_io) {
        *ctrl_io = ctrl;
        *dt_io = dt;
    }
    free(y);
    free(aux);
    st->t = t;
    if (ntrace) *ntrace = nt;
    return rc;
}

/* ---------------------------------------------------------------------------
 * Diagnostics: sum of c over all cells (plain sequential sum), and the
 * largest |sum_a phi_a - 1|, min and max of phi.
 * ------------------------------------------------------------------------- */
double pfo_sum_c(const pfo_params *P, const double *u) {
    long long V = ncells(P);
    double s = 0.0;
    if (!P->with_c) return 0.0;
    for (long long i = 0; i < V; ++i) s = s + u[(long long)P->n_phi * V + i];
    return s;
}

void pfo_phi_stats(const pfo_params *P, const double *u, double *max_sum_dev, double *pmin,
                   double *pmax) {
    long long V = ncells(P);
    double dev = 0.0, lo = INFINITY, hi = -INFINITY;
    for (long long i = 0; i < V; ++i) {
        double s = 0.0;
        for (int a = 0; a < P->n_phi; ++a) {
            double p = u[(long long)a * V + i];
            s = s + p;
            if (p < lo) lo = p;
            if (p > hi) hi = p;
        }
        if (fabs(s - 1.0) > dev) dev = fabs(s - 1.0);
    }
    *max_sum_dev = dev; *pmin = lo; *pmax = hi;
}

/* ---------------------------------------------------------------------------
 * Discrete free energy F_h (eqs. energy, wterm) used only to pin the
 * variational derivative by brute force: gradient products over the faces
 * (each face once), the pair potential per cell, and f = sum_a phi_a g_a(c_a)
 * with the KKS phase concentrations.  The obstacle's infinite branch is not
 * evaluated (the caller stays on the simplex or differentiates the finite
 * branch only).  Returns sum_i [a_i + w_i + f_i] dx^d.
 * ------------------------------------------------------------------------- */
double pfo_energy(const pfo_params *P, const double *u) {
    long long V = ncells(P);
    int N = P->n_phi;
    double dV = pow(P->dx, P->dim);
    double Etot = 0.0;
    for (long long i = 0; i < V; ++i) {
        long long nb[6];
        int nnb = neighbours(P, i, nb);
        double e = 0.0;
        /* gradient term over the "+" faces of cell i (x+, y+, z+) */
        for (int k = 1; k < nnb; k += 2) {
            long long j = nb[k];
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < a; ++b) {
                    double ga = (u[(long long)a * V + j] - u[(long long)a * V + i]) / P->dx;
                    double gb = (u[(long long)b * V + j] - u[(long long)b * V + i]) / P->dx;
                    e -= pair_A(P, a, b) * ga * gb;
                }
        }
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < a; ++b)
                e += pair_B(P, a, b) * u[(long long)a * V + i] * u[(long long)b * V + i];
        if (P->with_c) {
            /* phase concentrations from c = sum phi_a c_a and equal dg/dc */
            double num = u[(long long)N * V + i], den = 0.0;
            for (int a = 0; a < N; ++a) {
                int t = P->type_of[a];
                num -= u[(long long)a * V + i] * P->c0[t];
                den += u[(long long)a * V + i] / P->k[t];
            }
            double mu = num / den;
            for (int a = 0; a < N; ++a) {
                int t = P->type_of[a];
                double ca = P->c0[t] + mu / P->k[t];
                e += u[(long long)a * V + i] * 0.5 * P->k[t] * (ca - P->c0[t]) * (ca - P->c0[t]);
            }
        }
        Etot += e * dV;
    }
    return Etot;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int pfo_num_threads(void) { return omp_get_max_threads(); }
