// pf_api.cpp -- host engine and C-ABI of libpf (see include/pf.h).
//
// The engine owns the device state vectors, sequences the fused stage kernels
// of each integrator (Sec. 3.2 of Seiz & Takaki, arXiv 2601.16522), runs the
// adaptive loop with the error norm and PID controller of Sec. 3.3 and keeps
// the time in FP64.  Every arithmetic step on field data runs in the kernels
// of pf_kernels.hip; the host only computes scalar coefficients.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "pf_internal.h"

using namespace pf;

namespace {

constexpr int NBUF = 7;
constexpr int RES_DIAG = 0, RES_NORM = 8, RES_LEN = 16;
constexpr double PI = 3.14159265358979323846;

// Controller state (pf_controller of the C-ABI): bias b, accepted-history
// length and the last two accepted scaled errors and steps.
inline pf_controller ctrl_initial() {
    pf_controller c;
    c.b = 0.9;
    c.nhist = 0;
    c.E1 = c.E2 = c.h1 = c.h2 = 0.0;
    return c;
}

struct Pending {
    unsigned mask;
    hipEvent_t e0, e1;
    int count;  // launches between the two events
};

enum Family : unsigned {
    FAM_STAGE = 1u << 0,
    FAM_EST = 1u << 1,
    FAM_RED = 1u << 2,
    FAM_RKL2 = 1u << 3,
    FAM_FE = 1u << 4,
};

}  // namespace

struct pf_sim {
    int dim, nx, ny, nz, N, T, with_c, ssp_s;
    pf_precision prec;
    double dx, W;
    std::vector<int> type_of;
    std::vector<double> gamma, mob, k, c0, D;
    int walls = 0, cfix = 0;  // boundaries (pf_params bc / c_fixed as bit masks)
    double cbc[6] = {0, 0, 0, 0, 0, 0};
    int F;
    long long V;
    size_t esz;
    hipStream_t stream = nullptr;
    void *buf[NBUF] = {nullptr};
    int cur = 0;
    bool have_fields = false;
    void *dparams = nullptr;
    KConsts<float> kf{};
    KConsts<double> kd{};
    double *red = nullptr;
    long long *redn = nullptr;
    int red_cap = 0;
    // pinned, coherent host memory for scalar results: [RES_DIAG, +5) the
    // diagnostics, [RES_NORM, +4) the error norm (sum, count, norm, sequence)
    double *hres = nullptr;
    double *hres_dev = nullptr;  // the same memory as the device addresses it
    double res_seq = 0.0;        // sequence number of the last norm result
    double t = 0.0;
    pf_controller ctrl = ctrl_initial();
    double dt_next = 0.0;   // controller proposal carried between pf_run_to calls
    std::vector<double> trace;
    std::string err;
    int tx = 64, zchunk = 16;
    int zchunk2 = 32;        // z extent of the fused RKL2 stage pairs (3D)
    int groups_min = 1;      // least buffer groups per state vector (pf_set_field_groups)
    // sparse phase storage (pf_set_sparse_storage): slots per cell (0: dense),
    // byte offset of the id words in a buffer, device count of cut cells
    int n_p = 0;
    unsigned long long ids_off = 0;
    unsigned long long *dcut = nullptr;
    int fuse = 1;            // RKL2 inner stages per launch (2: fused pairs, where built)
    int r0rc = 0;            // 3D RKL2 inner stages recompute R0 from u0 (pf_set_r0_recompute)
    int inner_launches = 0;  // launches of the last step's inner-stage interval
    bool timing = false;
    unsigned timing_mask = 0;  // families recorded while timing
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double fam_ms[5] = {0, 0, 0, 0, 0};
    long long fam_n[5] = {0, 0, 0, 0, 0};
    pf_stats st{};
};

namespace {

pf_status fail(pf_sim *s, pf_status code, const char *fmt, ...) {
    if (s) {
        char b[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(b, sizeof b, fmt, ap);
        va_end(ap);
        s->err = b;
    }
    return code;
}

#define HIPCHK(s, expr)                                                                 \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail((s), PF_EHIP, "%s: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

size_t state_bytes(const pf_sim *s) { return (size_t)s->F * (size_t)s->V * s->esz; }

// Bytes of one work buffer: a dense vector, or with sparse phase storage the
// larger of a dense vector (R0, RHS) and a sparse one (c, n_p value planes,
// then the id words at ids_off).
size_t buf_bytes(const pf_sim *s) {
    if (s->n_p <= 0) return state_bytes(s);
    return std::max(state_bytes(s), (size_t)s->ids_off + 4 * (size_t)s->V);
}

// Buffer-group mask of the state vectors of a stage (y1, y2, u0 and, except
// for the RHS kind, out) under sparse phase storage.
unsigned sparse_mask(const pf_sim *s, int kind) {
    if (s->n_p <= 0) return 0u;
    return kind == K_RHS ? 0x7u : 0x17u;
}

// Buffer groups of the handle's state vectors: the fewest that address them,
// or more when pf_set_field_groups asked for more.
int sim_groups(const pf_sim *s) {
    int ng = std::max(field_groups_needed(s->N, s->V, (int)s->esz), s->groups_min);
    if (s->n_p > 0) ng = std::max(ng, field_groups_needed(SPMAX, s->V, (int)s->esz));
    return ng;
}

pf_status ensure_buf(pf_sim *s, int i) {
    if (!s->buf[i]) {
        if (hipMalloc(&s->buf[i], buf_bytes(s)) != hipSuccess) {
            s->buf[i] = nullptr;
            return fail(s, PF_ENOMEM, "hipMalloc of %zu bytes failed", buf_bytes(s));
        }
    }
    return PF_OK;
}

// Work buffer number k (0-based) other than the current state.
int work_index(const pf_sim *s, int k) {
    int idx = 0;
    for (int i = 0; i < NBUF; ++i) {
        if (i == s->cur) continue;
        if (idx == k) return i;
        ++idx;
    }
    return -1;
}

void tiles(const pf_sim *s, int &ntx, int &nty, int &nzc, int &ntiles, int &nblocks) {
    const int tx = s->tx, ty = tile_rows(s->dim, s->N);
    ntx = (s->nx + tx - 1) / tx;
    nty = (s->ny + ty - 1) / ty;
    nzc = s->dim == 3 ? (s->nz + s->zchunk - 1) / s->zchunk : 1;
    ntiles = ntx * nty * nzc;
    nblocks = (ntiles + 7) / 8 * 8;
}

pf_status ensure_red(pf_sim *s, int n) {
    if (n <= s->red_cap) return PF_OK;
    if (s->red) hipFree(s->red);
    if (s->redn) hipFree(s->redn);
    s->red = nullptr;
    s->redn = nullptr;
    if (hipMalloc(&s->red, sizeof(double) * 5 * (size_t)n) != hipSuccess ||
        hipMalloc(&s->redn, sizeof(long long) * (size_t)n) != hipSuccess) {
        s->red_cap = 0;
        return fail(s, PF_ENOMEM, "reduction buffers");
    }
    s->red_cap = n;
    return PF_OK;
}

hipEvent_t get_event(pf_sim *s) {
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

// Timing records one event pair around a run of back-to-back launches of one
// family (the inner stages of a step, the stages of a fixed-step run, one
// estimator launch), not around every launch, so that the events add no gap
// between the kernels they measure.
// fam: the families whose intervals the event bounds; it is recorded only when
// one of them is enabled.
hipEvent_t mark(pf_sim *s, unsigned fam) {
    if (!s->timing || !(s->timing_mask & fam)) return nullptr;
    hipEvent_t e = get_event(s);
    hipEventRecord(e, s->stream);
    return e;
}

void add_interval(pf_sim *s, unsigned mask, hipEvent_t e0, hipEvent_t e1, int count) {
    if (!s->timing || !e0 || !e1 || count <= 0) return;
    s->pending.push_back(Pending{mask, e0, e1, count});
}

void begin_timed(pf_sim *s, unsigned mask, Pending &p) {
    p.mask = mask;
    p.count = 1;
    p.e0 = p.e1 = nullptr;
    if (!s->timing || !(s->timing_mask & mask)) return;
    p.e0 = get_event(s);
    p.e1 = get_event(s);
    hipEventRecord(p.e0, s->stream);
}

void end_timed(pf_sim *s, Pending &p) {
    if (!s->timing || !p.e0) return;
    hipEventRecord(p.e1, s->stream);
    s->pending.push_back(p);
}

void collect_timing(pf_sim *s) {
    if (s->pending.empty()) return;
    hipStreamSynchronize(s->stream);
    // an event may close one interval and open the next: return each event to
    // the pool once
    std::vector<hipEvent_t> seen;
    for (auto &p : s->pending) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, p.e0, p.e1);
        for (int f = 0; f < 5; ++f)
            if (p.mask & (1u << f)) {
                s->fam_ms[f] += ms;
                s->fam_n[f] += p.count;
            }
        seen.push_back(p.e0);
        seen.push_back(p.e1);
    }
    std::sort(seen.begin(), seen.end());
    seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
    for (auto e : seen) s->pool.push_back(e);
    s->pending.clear();
}

// ---------------------------------------------------------------------------
// Constants (Sec. 2): A = 4 W gamma / pi, B = 4 gamma / (pi W), L = pi M / (4 W)
// ---------------------------------------------------------------------------
template <typename T>
void fill_kconsts(const DevParams<T> &P, KConsts<T> &K) {
    std::memset(&K, 0, sizeof K);
    K.nx = P.nx; K.ny = P.ny; K.nz = P.nz;
    K.with_c = P.with_c; K.n_types = P.n_types; K.uniform = P.uniform;
    K.walls = P.walls; K.cfix = P.cfix;
    for (int f = 0; f < 6; ++f) K.cbc[f] = P.cbc[f];
    K.V = P.V; K.idx2 = P.idx2;
    for (int a = 0; a < NMAX; ++a) {
        K.c0[a] = P.c0[a]; K.ik[a] = P.ik[a]; K.Dk[a] = P.Dk[a];
        K.hik[a] = P.hik[a]; K.k2[a] = P.k2[a];
    }
}

template <typename T>
const KConsts<T> &kconsts(const pf_sim *s);
template <>
const KConsts<float> &kconsts<float>(const pf_sim *s) { return s->kf; }
template <>
const KConsts<double> &kconsts<double>(const pf_sim *s) { return s->kd; }

template <typename T>
void fill_params(const pf_sim *s, DevParams<T> &P) {
    std::memset(&P, 0, sizeof P);
    P.nx = s->nx;
    P.ny = s->ny;
    P.nz = s->nz;
    P.n_phi = s->N;
    P.with_c = s->with_c;
    P.n_types = s->T;
    P.V = s->V;
    P.idx2 = (T)(1.0 / (s->dx * s->dx));
    for (int a = 0; a < s->N; ++a) {
        const int ta = s->type_of[a];
        for (int b = 0; b < s->N; ++b) {
            const int tb = s->type_of[b];
            const double g = s->gamma[ta * s->T + tb];
            const double m = s->mob[ta * s->T + tb];
            P.A[a * NMAX + b] = (T)(4.0 * s->W * g / PI);
            P.B[a * NMAX + b] = (T)(4.0 * g / (PI * s->W));
            P.L[a * NMAX + b] = (T)(PI * m / (4.0 * s->W));
        }
        const double ik = 1.0 / s->k[ta];
        P.c0[a] = (T)s->c0[ta];
        P.ik[a] = (T)ik;
        P.Dk[a] = (T)(s->D[ta] * ik);
        P.k2[a] = (T)(2.0 * s->k[ta]);
        P.hik[a] = (T)(0.5 * ik);
        P.tphi[a] = ta;
    }
    for (int t = 0; t < s->T; ++t) {
        const double ik = 1.0 / s->k[t];
        P.k2t[t] = (T)(2.0 * s->k[t]);
        P.hikt[t] = (T)(0.5 * ik);
        P.c0t[t] = (T)s->c0[t];
        P.ikt[t] = (T)ik;
        P.Dkt[t] = (T)(s->D[t] * ik);
    }
    int uni = 1;
    for (int a = 0; a < s->N; ++a)
        for (int b = 0; b < s->N; ++b) {
            if (a == b) continue;
            uni &= P.A[a * NMAX + b] == P.A[1] && P.B[a * NMAX + b] == P.B[1] &&
                   P.L[a * NMAX + b] == P.L[1];
        }
    P.uniform = uni;
    P.walls = s->walls;
    P.cfix = s->cfix;
    for (int f = 0; f < 6; ++f) P.cbc[f] = (T)s->cbc[f];
}

// Stable Euler step (Sec. 3.2, Gershgorin estimates of the two-phase system):
//   lambda_phi = Mx gx (4d/dx^2 - 1/W^2) + [c, dc0 != 0] (pi Mx/(8W)) kx (dc0^2 + |dc0|)
//   lambda_c   = 4 d Dx / dx^2 (1 + |dc0|/2),   dt_e = 2 / max.
double stable_dt(const pf_sim *s) {
    const int T = s->T;
    double Mx = 0, gx = 0, kx = 0, Dx = 0, dc0 = 0;
    std::vector<int> used(T, 0);
    for (int a = 0; a < s->N; ++a) used[s->type_of[a]] = 1;
    for (int i = 0; i < T; ++i) {
        if (!used[i]) continue;
        kx = std::max(kx, s->k[i]);
        Dx = std::max(Dx, s->D[i]);
        for (int j = 0; j < T; ++j) {
            if (!used[j]) continue;
            Mx = std::max(Mx, s->mob[i * T + j]);
            gx = std::max(gx, s->gamma[i * T + j]);
            dc0 = std::max(dc0, std::fabs(s->c0[i] - s->c0[j]));
        }
    }
    const double idx2 = 1.0 / (s->dx * s->dx);
    double lam = Mx * gx * (4.0 * s->dim * idx2 - 1.0 / (s->W * s->W));
    if (s->with_c) {
        if (dc0 != 0.0) lam += (PI * Mx / (8.0 * s->W)) * kx * (dc0 * dc0 + dc0);
        const double lc = 4.0 * s->dim * Dx * idx2 * (1.0 + dc0 / 2.0);
        lam = std::max(lam, lc);
    }
    return 2.0 / lam;
}

// Exact output times (Sec. 5): the step from t towards t_end has size h unless
// the remainder is at most h (1 + 1e-10); then it is the remainder and the
// last one.  A remainder at most 1e-12 h means t_end is reached (false).
bool clip_step(double t, double t_end, double h, double &h_use, bool &last) {
    const double rem = t_end - t;
    // an infinite step (dt_e is infinite without mobility and diffusion, where
    // the right-hand side vanishes) is clipped to the remainder like any step
    // that would pass t_end
    if (rem <= 1e-12 * (std::isinf(h) ? rem : h)) return false;
    last = rem <= h * (1.0 + 1e-10);
    h_use = last ? rem : h;
    return true;
}

// Smallest odd stage count inside the exact RKL stability bound times 0.9.
int stage_count(int order, double dt, double dte) {
    if (!(dt > 0.0) || !(dte > 0.0)) return -1;
    const double h = 0.9 * dte;
    for (int s = order == 1 ? 1 : 3; s < 1000000; s += 2) {
        const double lim = order == 1 ? h * ((double)s * s + s) / 2.0
                                      : h * ((double)s * s + s - 2.0) / 4.0;
        if (dt <= lim) return s;
    }
    return -1;
}

// RKL coefficients (Meyer et al. 2012/2014), stage j of s.
double rkl2_b(int j) {
    if (j < 3) return 1.0 / 3.0;
    return ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
}

void rkl_coeffs(int order, int s, int j, double &mu, double &nu, double &mut, double &gam) {
    if (order == 1) {
        const double w1 = 2.0 / ((double)s * s + s);
        if (j == 1) {
            mu = nu = gam = 0.0;
            mut = w1;
            return;
        }
        mu = (2.0 * j - 1.0) / j;
        nu = (1.0 - j) / j;
        mut = w1 * mu;
        gam = 0.0;
        return;
    }
    const double w1 = 4.0 / ((double)s * s + s - 2.0);
    if (j == 1) {
        mu = nu = gam = 0.0;
        mut = rkl2_b(1) * w1;
        return;
    }
    mu = (2.0 * j - 1.0) / j * (rkl2_b(j) / rkl2_b(j - 1));
    nu = -(j - 1.0) / j * (rkl2_b(j) / rkl2_b(j - 2));
    mut = mu * w1;
    gam = -(1.0 - rkl2_b(j - 1)) * mut;
}

int method_order(int integ) {
    switch (integ) {
    case PF_FEULER: return 1;
    case PF_SSP_S2: return 2;
    case PF_SSP_10_4: return 4;
    case PF_RKL1: return 1;
    default: return 2;
    }
}

// PID controller of Sec. 3.3 (Soederlind), bias b in [0.1, 0.98].
double ctrl_update(pf_controller &c, int order, double e, double h, bool &accept) {
    const double k1 = 1.25, k2 = 0.5, k3 = -0.6, k4 = 0.25, k5 = 0.0;
    const double p1 = order + 1.0;
    const bool finite = std::isfinite(e);
    const bool acc = finite && e < 1.0;
    double F;
    double E = e / c.b;
    if (E < 1e-12) E = 1e-12;
    if (!finite) {
        F = 0.0;
    } else {
        double prod = std::pow(E, -k1);
        if (c.nhist >= 1) prod = prod * std::pow(c.E1, -k2);
        if (c.nhist >= 2) prod = prod * std::pow(c.E2, -k3);
        F = std::pow(prod, 1.0 / p1);
        if (c.nhist >= 1) F = F * std::pow(h / c.h1, k4);
        if (c.nhist >= 2) F = F * std::pow(c.h1 / c.h2, k5);
        if (!acc && F > 1.0) {
            const double en = e < 1e-12 ? 1e-12 : e;
            F = std::pow(en, -k1 / p1);
        }
    }
    const double hn = h * (1.0 + 5.0 * std::atan((F - 1.0) / 5.0));
    if (acc) {
        c.E2 = c.E1;
        c.h2 = c.h1;
        c.E1 = E;
        c.h1 = h;
        if (c.nhist < 2) c.nhist++;
        c.b = std::min(std::sqrt(c.b), 0.98);
    } else {
        c.b = std::max(c.b * c.b, 0.1);
    }
    accept = acc;
    return hn;
}

// ---------------------------------------------------------------------------
// Kernel launches
// ---------------------------------------------------------------------------
template <typename T>
T *bp(pf_sim *s, int i) { return i < 0 ? nullptr : (T *)s->buf[i]; }

template <typename T>
pf_status stage(pf_sim *s, int kind, const T *y1, const T *y2, const T *u0, const T *r0, T *out,
                T *out2, double a, double b, double c, double d, double e, double f,
                unsigned fam, double a2 = 0.0) {
    StageArgs<T> A;
    std::memset(&A, 0, sizeof A);
    A.K = kconsts<T>(s);
    A.P = (const DevParams<T> *)s->dparams;
    A.y1 = y1;
    A.y2 = y2;
    A.u0 = u0;
    A.r0 = r0;
    A.out = out;
    A.out2 = out2;
    set_field_bases(A, s->N, s->V, s->groups_min, sparse_mask(s, kind));
    A.n_p = s->n_p;
    A.ids_off = s->ids_off;
    A.cut = s->dcut;
    A.kind = kind;
    A.a = (T)a; A.b = (T)b; A.c = (T)c; A.d = (T)d; A.e = (T)e; A.f = (T)f;
    A.a2 = (T)a2;
    int ntx, nty, nzc, ntiles, nblocks;
    tiles(s, ntx, nty, nzc, ntiles, nblocks);
    A.tx = s->tx;
    A.ty = tile_rows(s->dim, s->N);
    A.zchunk = s->zchunk;
    A.ntx = ntx;
    A.nty = nty;
    A.nzc = nzc;
    A.ntiles = ntiles;
    (void)fam;
    hipError_t err = launch_stage<T>(s->dim, s->N, A, nblocks, s->stream);
    if (err != hipSuccess) return fail(s, PF_EHIP, "stage kernel launch: %s", hipGetErrorString(err));
    return PF_OK;
}

// Whether RKL2 inner stages can recompute R0 from u0 (K_RKL2_RC): periodic 3D
// grids in dense storage, where the kernel is built.
bool rc_ok(const pf_sim *s) {
    return s->dim == 3 && s->walls == 0 && s->n_p == 0 && rkl2_rc_built((int)s->esz, s->N);
}

// Whether the fused RKL2 stage-pair kernel is built for the simulation:
// periodic grids; in 2D with vectors in one buffer group and the kernel's LDS
// within one workgroup's, in 3D where its two z windows fit the registers.
bool pair_ok(const pf_sim *s) {
    if (s->walls != 0 || s->n_p > 0) return false;
    if (s->dim == 2) return sim_groups(s) == 1 && rkl2_pair_fits((int)s->esz, s->N);
    return rkl2_pair3_built((int)s->esz, s->N);
}

// RKL2 stages j and j + 1 in one launch: y1 = Y_{j-1}, y2 = Y_{j-2}, out = Y_j,
// out2 = Y_{j+1}; c1, c2: the K_RKL2 coefficients of the two stages.
template <typename T>
pf_status stage_pair(pf_sim *s, const T *y1, const T *y2, const T *u0, const T *r0, T *out, T *out2,
                     const double c1[6], const double c2[6]) {
    StageArgs<T> A;
    std::memset(&A, 0, sizeof A);
    A.K = kconsts<T>(s);
    A.P = (const DevParams<T> *)s->dparams;
    A.y1 = y1;
    A.y2 = y2;
    A.u0 = u0;
    A.r0 = r0;
    A.out = out;
    A.out2 = out2;
    set_field_bases(A, s->N, s->V, s->groups_min);
    A.kind = K_RKL2_PAIR;
    A.a = (T)c1[0]; A.b = (T)c1[1]; A.c = (T)c1[2]; A.d = (T)c1[3]; A.e = (T)c1[4]; A.f = (T)c1[5];
    A.a2 = (T)c2[0]; A.b2 = (T)c2[1]; A.c2 = (T)c2[2]; A.d2 = (T)c2[3]; A.e2 = (T)c2[4]; A.f2 = (T)c2[5];
    const bool d3 = s->dim == 3;
    A.tx = d3 ? P3_TX : P2_TX;
    A.ty = d3 ? P3_TY : P2_TY;
    A.zchunk = d3 ? s->zchunk2 : 1;
    A.ntx = (s->nx + A.tx - 1) / A.tx;
    A.nty = (s->ny + A.ty - 1) / A.ty;
    A.nzc = d3 ? (s->nz + A.zchunk - 1) / A.zchunk : 1;
    A.ntiles = A.ntx * A.nty * A.nzc;
    const int nblocks = (A.ntiles + 7) / 8 * 8;
    hipError_t err = launch_stage<T>(s->dim, s->N, A, nblocks, s->stream);
    if (err != hipSuccess) return fail(s, PF_EHIP, "stage-pair kernel launch: %s", hipGetErrorString(err));
    return PF_OK;
}

// Sommeijer-type estimate (kind 0) or embedded estimate (kind 1) -> norm on host.
// Waits for the norm kernel's result: it writes the result and then sequence
// number seq into the coherent host buffer, which is polled here (cheaper than
// a stream synchronisation for one scalar per adaptive step).  The stream is
// queried every few thousand polls, so a stream that drains or fails without
// the number ends the wait with an error instead of a hang.
pf_status wait_result(pf_sim *s, double seq) {
    volatile const double *flag = s->hres + RES_NORM + 3;
    for (unsigned long it = 1;; ++it) {
        if (*flag == seq) break;
        if ((it & 4095u) == 0) {
            const hipError_t q = hipStreamQuery(s->stream);
            if (q == hipSuccess) {
                if (*flag == seq) break;
                return fail(s, PF_EHIP, "norm result missing after the stream drained");
            }
            if (q != hipErrorNotReady) return fail(s, PF_EHIP, "stream: %s", hipGetErrorString(q));
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return PF_OK;
}

// Partial sums of an error norm: one per tile for the estimate of Sec. 3.3
// (kind 0), one per block of the grid-stride embedded estimate (kind 1).
constexpr int EMBED_BLOCKS = 1024;
int norm_partials(const pf_sim *s, int kind) {
    int ntx, nty, nzc, ntiles, nblocks;
    tiles(s, ntx, nty, nzc, ntiles, nblocks);
    return kind == 0 ? ntiles : EMBED_BLOCKS;
}

// The estimate and its norm with the partial sums in red / redn (at least
// norm_partials(s, kind) entries each); timed: record the timing events (the
// allocation-free path records none, since events may be created on demand).
template <typename T>
pf_status error_norm_with(pf_sim *s, int kind, double dt, const T *uold, const T *unew, const T *aux,
                          const pf_tol &tol, double *red, long long *redn, bool timed, double *norm,
                          long long *ndof) {
    int ntx, nty, nzc, ntiles, nblocks;
    tiles(s, ntx, nty, nzc, ntiles, nblocks);
    const int nred = norm_partials(s, kind);
    const bool was_timing = s->timing;
    if (!timed) s->timing = false;
    pf_status rc = PF_OK;
    Pending p;
    if (kind == 0) {
        StageArgs<T> A;
        std::memset(&A, 0, sizeof A);
        A.K = kconsts<T>(s);
        A.P = (const DevParams<T> *)s->dparams;
        A.y1 = unew;
        A.u0 = uold;
        A.r0 = aux;
        set_field_bases(A, s->N, s->V, s->groups_min);
        A.kind = K_EST;
        A.red = red;
        A.redn = redn;
        A.r_phi = (T)tol.r_phi; A.a_phi = (T)tol.a_phi;
        A.r_c = (T)tol.r_c; A.a_c = (T)tol.a_c;
        A.dt6 = (T)(6.0 * dt);
        A.hdt = (T)(dt / 2.0);
        A.tx = s->tx; A.ty = tile_rows(s->dim, s->N); A.zchunk = s->zchunk;
        A.ntx = ntx; A.nty = nty; A.nzc = nzc; A.ntiles = ntiles;
        begin_timed(s, FAM_EST, p);
        hipError_t err = launch_stage<T>(s->dim, s->N, A, nblocks, s->stream);
        if (err != hipSuccess) rc = fail(s, PF_EHIP, "estimator launch: %s", hipGetErrorString(err));
        end_timed(s, p);
    } else {
        begin_timed(s, FAM_EST, p);
        hipError_t err = launch_embed_est<T>((const DevParams<T> *)s->dparams, s->N, s->with_c, s->V,
                                             unew, aux, uold, (T)tol.r_phi, (T)tol.a_phi,
                                             (T)tol.r_c, (T)tol.a_c, red, redn, nred, s->stream);
        if (err != hipSuccess) rc = fail(s, PF_EHIP, "embedded estimator launch: %s", hipGetErrorString(err));
        end_timed(s, p);
    }
    if (!rc) {
        begin_timed(s, FAM_RED, p);
        s->res_seq += 1.0;
        const hipError_t err = launch_finalize_norm(red, redn, nred, s->hres_dev + RES_NORM, s->res_seq,
                                                    s->stream);
        if (err != hipSuccess) rc = fail(s, PF_EHIP, "norm launch: %s", hipGetErrorString(err));
        end_timed(s, p);
    }
    s->timing = was_timing;
    if (rc) return rc;
    if ((rc = wait_result(s, s->res_seq))) return rc;
    *norm = s->hres[RES_NORM + 2];
    if (ndof) *ndof = (long long)s->hres[RES_NORM + 1];
    s->st.rhs_evals += kind == 0 ? 1 : 0;
    return PF_OK;
}

template <typename T>
pf_status error_norm(pf_sim *s, int kind, double dt, const T *uold, const T *unew, const T *aux,
                     const pf_tol &tol, double *norm, long long *ndof) {
    pf_status rc = ensure_red(s, std::max(norm_partials(s, kind), EMBED_BLOCKS));
    if (rc) return rc;
    return error_norm_with<T>(s, kind, dt, uold, unew, aux, tol, s->red, s->redn, true, norm, ndof);
}

// ---------------------------------------------------------------------------
// Integrator steps.  The state is buffer `cur`; work buffers are allocated on
// demand.  On return *res is the buffer holding u^{n+1}, *aux the buffer with
// rhs(u^n) (RKL, corrected for RKL2) or the embedded solution (SSP(s)2), or -1.
// The state buffer is never written (keep_u) unless the RKL1 three-buffer
// scheme of Alg. sts1 is requested for a fixed step.
// ---------------------------------------------------------------------------
template <typename T>
pf_status do_step_impl(pf_sim *s, int integ, int nst, double dt, bool want_aux, int *res, int *aux,
                       hipEvent_t *e_inner);

// One step with its stage kernels timed as a run (see mark()); timed == false
// leaves the timing to the caller (a fixed forward-Euler run times the whole
// sequence of steps).
template <typename T>
pf_status do_step(pf_sim *s, int integ, int nst, double dt, bool want_aux, int *res, int *aux,
                  bool timed = true) {
    const long long st0 = s->st.stages;
    const unsigned fam = FAM_STAGE | (integ == PF_FEULER ? FAM_FE : 0u);
    hipEvent_t e0 = timed ? mark(s, fam) : nullptr, ei = nullptr;
    pf_status rc = do_step_impl<T>(s, integ, nst, dt, want_aux, res, aux, timed ? &ei : nullptr);
    if (rc || !timed) return rc;
    hipEvent_t e1 = mark(s, fam | (integ == PF_RKL2 ? FAM_RKL2 : 0u));
    const int n = (int)(s->st.stages - st0);
    add_interval(s, FAM_STAGE | (integ == PF_FEULER ? FAM_FE : 0u), e0, e1, n);
    if (integ == PF_RKL2) add_interval(s, FAM_RKL2, ei, e1, s->inner_launches);
    return PF_OK;
}

template <typename T>
pf_status do_step_impl(pf_sim *s, int integ, int nst, double dt, bool want_aux, int *res, int *aux,
                       hipEvent_t *e_inner) {
    const int U = s->cur;
    *aux = -1;
    auto W = [&](int k) { return work_index(s, k); };
    pf_status rc;
    int need = 1;
    if (integ == PF_SSP_S2) need = 2;
    else if (integ == PF_SSP_10_4) need = 3;
    else if (integ == PF_RKL1) need = want_aux ? 4 : 2;
    const bool pairs = integ == PF_RKL2 && s->fuse == 2 && pair_ok(s);
    if (integ == PF_RKL2) need = pairs ? 5 : 4;
    for (int k = 0; k < need; ++k)
        if ((rc = ensure_buf(s, W(k)))) return rc;
    const T *u = bp<T>(s, U);
    switch (integ) {
    case PF_FEULER: {
        rc = stage<T>(s, K_EULER, u, nullptr, nullptr, nullptr, bp<T>(s, W(0)), nullptr, dt, 0, 0, 0,
                      0, 0, FAM_FE);
        if (rc) return rc;
        s->st.rhs_evals++;
        s->st.stages++;
        *res = W(0);
        return PF_OK;
    }
    case PF_SSP_S2: {
        const int ns = nst;
        if (ns < 2) return fail(s, PF_EINVAL, "SSP(s)2 needs s >= 2");
        int q1 = U;
        int pp[2] = {W(0), W(1)};
        int which = 0;
        for (int i = 1; i <= ns - 1; ++i) {
            const int dst = pp[which];
            // Alg. ssp2: q3 = q1 + dt (rhs(q1) / (s - 1))
            rc = stage<T>(s, K_EULER, bp<T>(s, q1), nullptr, nullptr, nullptr, bp<T>(s, dst), nullptr,
                          dt, (double)(ns - 1), 0, 0, 0, 0, 0);
            if (rc) return rc;
            q1 = dst;
            which ^= 1;
            s->st.rhs_evals++;
            s->st.stages++;
        }
        const int dst = pp[which];
        rc = stage<T>(s, K_SSP2_FINAL, bp<T>(s, q1), nullptr, u, nullptr, bp<T>(s, dst), nullptr,
                      (double)(ns - 1), dt, (double)ns, 0, 0, 0, 0);
        if (rc) return rc;
        s->st.rhs_evals++;
        s->st.stages++;
        *res = dst;
        *aux = q1;  // embedded first-order solution Y_{s-1}
        return PF_OK;
    }
    case PF_SSP_10_4: {
        int q1 = U;
        int pp[2] = {W(0), W(1)};
        const int Q2 = W(2);
        int which = 0;
        const T *q2 = u;
        for (int i = 1; i <= 9; ++i) {
            const int dst = pp[which];
            if (i == 5) {
                rc = stage<T>(s, K_SSP104_S5, bp<T>(s, q1), nullptr, q2, nullptr, bp<T>(s, dst),
                              bp<T>(s, Q2), dt / 6.0, 1.0 / 25.0, 9.0 / 25.0, 15.0, 5.0, 2.0 / 5.0, 0);
                q2 = bp<T>(s, Q2);
            } else {
                rc = stage<T>(s, K_EULER, bp<T>(s, q1), nullptr, nullptr, nullptr, bp<T>(s, dst),
                              nullptr, dt / 6.0, 0, 0, 0, 0, 0, 0);
            }
            if (rc) return rc;
            q1 = dst;
            which ^= 1;
            s->st.rhs_evals++;
            s->st.stages++;
        }
        const int dst = pp[which];
        // (the single-precision form reads u^n as y2 and uses c = 9/25)
        rc = stage<T>(s, K_SSP104_FINAL, bp<T>(s, q1), u, q2, nullptr, bp<T>(s, dst), nullptr,
                      3.0 / 5.0, dt / 10.0, 9.0 / 25.0, 0, 0, 0, 0);
        if (rc) return rc;
        s->st.rhs_evals++;
        s->st.stages++;
        *res = dst;
        *aux = q1;  // embedded solution: the tenth stage value Y_10 (second order)
        return PF_OK;
    }
    case PF_RKL1:
    case PF_RKL2: {
        const int order = integ == PF_RKL1 ? 1 : 2;
        const int ns = nst;
        if (ns < order) return fail(s, PF_EINVAL, "bad RKL stage count %d", ns);
        const bool second = order == 2;
        const bool keep_r0 = second || want_aux;
        // ring of three stage slots; slot 0 starts as u^{n,0}.  A fixed RKL1 step
        // is the three-buffer scheme of Alg. sts1 (u^{n,0} is overwritten by stage
        // 3, it is not read again); otherwise slot 0 is backed by a work buffer
        // from its first write on and u^{n,0} stays intact.
        const bool inplace = !second && !want_aux;
        const int R0 = keep_r0 ? W(3) : -1;
        // fused pairs read two ring slots and write two others: a ring of four
        const int NR = pairs ? 4 : 3;
        int slot[4] = {U, W(0), W(1), pairs ? W(4) : -1};
        const int slot0_store = inplace ? U : W(2);
        double mu, nu, mut, gam;
        rkl_coeffs(order, ns, 1, mu, nu, mut, gam);
        const double mut1 = mut;
        if (second) {
            rc = stage<T>(s, K_RKL2_FIRST, u, nullptr, nullptr, nullptr, bp<T>(s, slot[1]),
                          bp<T>(s, R0), mut1 * dt, 0, 0, 0, 0, 0, 0);
        } else {
            rc = stage<T>(s, K_EULER, u, nullptr, nullptr, nullptr, bp<T>(s, slot[1]),
                          keep_r0 ? bp<T>(s, R0) : nullptr, dt * mut1, 0, 0, 0, 0, 0, 0);
        }
        if (rc) return rc;
        s->st.rhs_evals++;
        s->st.stages++;
        // fused pairs: stage counts are odd, so the inner stages pair up; an
        // even count would run its first inner stage alone, ahead of the
        // timed inner interval, which holds pair launches only
        const int single_end = pairs ? ((ns - 1) % 2 ? 2 : 1) : ns;
        s->inner_launches = pairs ? (ns - 1) / 2 : ns - 1;
        if (e_inner && !pairs) *e_inner = mark(s, FAM_RKL2);
        for (int j = 2; j <= single_end; ++j) {
            const int jc = j % NR, jp = (j - 1) % NR, jpp = (j - 2) % NR;
            if (jc == 0) slot[0] = slot0_store;
            rkl_coeffs(order, ns, j, mu, nu, mut, gam);
            if (second && s->r0rc && rc_ok(s)) {
                // R0 recomputed from u^{n,0} with the first stage's mut_1 dt
                rc = stage<T>(s, K_RKL2_RC, bp<T>(s, slot[jp]), bp<T>(s, slot[jpp]), u, nullptr,
                              bp<T>(s, slot[jc]), nullptr, (1.0 - mu) - nu, mu, nu, dt, mut, gam,
                              FAM_RKL2, mut1 * dt);
            } else if (second) {
                rc = stage<T>(s, K_RKL2, bp<T>(s, slot[jp]), bp<T>(s, slot[jpp]), u, bp<T>(s, R0),
                              bp<T>(s, slot[jc]), nullptr, (1.0 - mu) - nu, mu, nu, dt, mut, gam,
                              FAM_RKL2);
            } else {
                rc = stage<T>(s, K_RKL1, bp<T>(s, slot[jp]), bp<T>(s, slot[jpp]), nullptr, nullptr,
                              bp<T>(s, slot[jc]), nullptr, mu, nu, dt * mut, 0, 0, 0, 0);
            }
            if (rc) return rc;
            s->st.rhs_evals++;
            s->st.stages++;
        }
        if (pairs) {
            if (e_inner && s->inner_launches > 0) *e_inner = mark(s, FAM_RKL2);
            for (int j = single_end + 1; j < ns; j += 2) {
                double c1[6], c2[6];
                rkl_coeffs(order, ns, j, mu, nu, mut, gam);
                c1[0] = (1.0 - mu) - nu; c1[1] = mu; c1[2] = nu; c1[3] = dt; c1[4] = mut; c1[5] = gam;
                rkl_coeffs(order, ns, j + 1, mu, nu, mut, gam);
                c2[0] = (1.0 - mu) - nu; c2[1] = mu; c2[2] = nu; c2[3] = dt; c2[4] = mut; c2[5] = gam;
                const int jc = j % NR, jn = (j + 1) % NR, jp = (j - 1) % NR, jpp = (j - 2) % NR;
                if (jc == 0 || jn == 0) slot[0] = slot0_store;
                rc = stage_pair<T>(s, bp<T>(s, slot[jp]), bp<T>(s, slot[jpp]), u, bp<T>(s, R0),
                                   bp<T>(s, slot[jc]), bp<T>(s, slot[jn]), c1, c2);
                if (rc) return rc;
                s->st.rhs_evals += 2;
                s->st.stages += 2;
            }
        }
        *res = slot[ns % NR];
        *aux = R0;
        return PF_OK;
    }
    default: return fail(s, PF_EINVAL, "unknown integrator %d", integ);
    }
}

template <typename T>
pf_status run_to_t(pf_sim *s, int integ, double t_end, const pf_tol *tol, double dt_fixed) {
    const double dte = stable_dt(s);
    s->trace.clear();
    pf_status rc;
    if (!tol) {
        if (!(dt_fixed > 0.0)) return fail(s, PF_EINVAL, "dt_fixed must be > 0");
        const bool fe = integ == PF_FEULER;
        hipEvent_t e_run = fe ? mark(s, FAM_STAGE | FAM_FE) : nullptr;
        const long long st_run = s->st.stages;
        for (;;) {
            double h;
            bool last;
            if (!clip_step(s->t, t_end, dt_fixed, h, last)) break;
            int ns = s->ssp_s;
            if (integ == PF_RKL1 || integ == PF_RKL2) ns = stage_count(integ == PF_RKL1 ? 1 : 2, h, dte);
            int res, aux;
            if ((rc = do_step<T>(s, integ, ns, h, false, &res, &aux, !fe))) return rc;
            s->cur = res;
            s->st.accepted++;
            s->trace.insert(s->trace.end(), {h, (double)ns, 0.0, 1.0});
            s->t = last ? t_end : s->t + h;
            s->st.last_dt = h;
        }
        if (fe) add_interval(s, FAM_STAGE | FAM_FE, e_run, mark(s, FAM_STAGE | FAM_FE),
                             (int)(s->st.stages - st_run));
        s->st.t = s->t;
        return PF_OK;
    }
    if (integ != PF_RKL1 && integ != PF_RKL2 && integ != PF_SSP_S2 && integ != PF_SSP_10_4)
        return fail(s, PF_EUNSUPPORTED, "adaptive stepping needs RKL1, RKL2, SSP(s)2 or SSP(10)4");
    const int order = method_order(integ);
    // the SSP schemes estimate the error with their embedded solutions
    const bool embedded = integ == PF_SSP_S2 || integ == PF_SSP_10_4;
    const double dtmax_ratio = tol->dt_max_over_dte > 0.0 ? tol->dt_max_over_dte : 200.0;
    double dtmax = dtmax_ratio * dte;
    if (integ == PF_SSP_S2) dtmax = std::min(dtmax, 0.9 * (s->ssp_s - 1) * dte);
    if (integ == PF_SSP_10_4) dtmax = std::min(dtmax, 0.9 * 6.0 * dte);
    // the controller (bias, accepted history, proposed step) carries over from
    // the previous pf_run_to of this handle; pf_init_fields resets it
    double dt = tol->dt0 > 0.0 ? tol->dt0 : (s->dt_next > 0.0 ? s->dt_next : 0.9 * dte);
    int nonfinite = 0;
    for (;;) {
        double h;
        bool last;
        if (!clip_step(s->t, t_end, std::min(dt, dtmax), h, last)) break;
        if (!last && std::isfinite(dte) && h < 1e-12 * dte)
            return fail(s, PF_EDTMIN, "adaptive step underflow (dt = %g)", h);
        int ns = s->ssp_s;
        if (integ == PF_SSP_10_4) ns = 10;
        else if (integ != PF_SSP_S2) ns = stage_count(order, h, dte);
        int res, aux;
        if ((rc = do_step<T>(s, integ, ns, h, true, &res, &aux))) return rc;
        double e;
        if ((rc = error_norm<T>(s, embedded ? 1 : 0, h, bp<T>(s, s->cur), bp<T>(s, res),
                                bp<T>(s, aux), *tol, &e, nullptr)))
            return rc;
        bool acc;
        const double hn = ctrl_update(s->ctrl, order, e, h, acc);
        s->trace.insert(s->trace.end(), {h, (double)ns, e, acc ? 1.0 : 0.0});
        s->st.last_err = e;
        if (acc) {
            s->cur = res;
            s->t = last ? t_end : s->t + h;
            s->st.accepted++;
            s->st.last_dt = h;
            nonfinite = 0;
        } else {
            s->st.rejected++;
            if (!std::isfinite(e) && ++nonfinite >= 3) {
                s->st.t = s->t;
                return fail(s, PF_ENONFINITE, "non-finite error norm three times in a row");
            }
        }
        dt = hn;
        s->dt_next = hn;
    }
    s->st.t = s->t;
    return PF_OK;
}

template <typename T>
pf_status upload(pf_sim *s, const double *phi, const double *c) {
    const long long V = s->V;
    std::vector<T> h((size_t)s->F * V);
    for (long long i = 0; i < (long long)s->N * V; ++i) h[i] = (T)phi[i];
    if (s->with_c) {
        const double *cc = c ? c : phi + (long long)s->N * V;
        for (long long i = 0; i < V; ++i) h[(long long)s->N * V + i] = (T)cc[i];
    }
    if (s->n_p > 0) {
        // dense into a work buffer, then packed into the state
        const int w = work_index(s, 0);
        if (pf_status rc = ensure_buf(s, w)) return rc;
        HIPCHK(s, hipMemcpyAsync(s->buf[w], h.data(), state_bytes(s), hipMemcpyHostToDevice, s->stream));
        HIPCHK(s, launch_pack_sparse<T>((const T *)s->buf[w], (T *)s->buf[s->cur], s->N, s->with_c, s->V,
                                        s->n_p, s->ids_off, s->dcut, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        return PF_OK;
    }
    HIPCHK(s, hipMemcpyAsync(s->buf[s->cur], h.data(), state_bytes(s), hipMemcpyHostToDevice,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return PF_OK;
}

template <typename T>
pf_status download(pf_sim *s, const void *dev, double *phi, double *c, bool sparse = false) {
    const long long V = s->V;
    std::vector<T> h((size_t)s->F * V);
    if (sparse) {  // a state in sparse storage: unpacked into a work buffer first
        const int w = work_index(s, 0);
        if (pf_status rc = ensure_buf(s, w)) return rc;
        HIPCHK(s, launch_unpack_sparse<T>((const T *)dev, (T *)s->buf[w], s->N, s->with_c, s->V, s->n_p,
                                          s->ids_off, s->stream));
        dev = s->buf[w];
    }
    HIPCHK(s, hipMemcpyAsync(h.data(), dev, state_bytes(s), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (phi)
        for (long long i = 0; i < (long long)s->N * V; ++i) phi[i] = (double)h[i];
    if (c && s->with_c)
        for (long long i = 0; i < V; ++i) c[i] = (double)h[(long long)s->N * V + i];
    return PF_OK;
}

#define DISPATCH(s, fn, ...) \
    ((s)->prec == PF_FP64 ? fn<double>(s, __VA_ARGS__) : fn<float>(s, __VA_ARGS__))

pf_status need_fields(pf_sim *s) {
    return s->have_fields ? PF_OK : fail(s, PF_ESTATE, "fields not initialised");
}

struct CkptHeader {
    char magic[8];
    int prec, F;
    long long V;
    double t, dt_next;
    double b, E1, E2, h1, h2;
    int nhist, pad;
    pf_stats st;
};

// Times the RKL2 inner-stage kernel (the dominant launch of the multi-stage
// integrators: one stencil vector and three plain vectors read, one written)
// for every candidate z extent and keeps the fastest.  Its four inputs are the
// current state and copies of it in three distinct work buffers (w[1..3]; the
// output goes to w[0]), so that caches see the traffic of a real stage; the
// candidates are timed in two interleaved passes and each keeps its faster
// time, which damps clock and queue noise between candidates.
template <typename T>
pf_status autotune_t(pf_sim *s, const int w[5], double &best, int &bzc, int &fuse, int &bzc2,
                     int &r0rc) {
    const int zcs3[7] = {4, 8, 16, 32, 64, 128, 256};
    const int ncand = s->dim == 3 ? 7 : 1;
    // fused pairs: one candidate in 2D, the z extents 8..128 in 3D
    const int zcp[5] = {8, 16, 32, 64, 128};
    const int npair = !pair_ok(s) ? 0 : (s->dim == 3 ? 5 : 1);
    // stages that recompute R0 (3D): the single-stage z extents again
    const int nrc = rc_ok(s) ? ncand : 0;
    const T *u = bp<T>(s, s->cur);
    for (int k = 1; k < 4; ++k)
        HIPCHK(s, hipMemcpyAsync(s->buf[w[k]], u, buf_bytes(s), hipMemcpyDeviceToDevice, s->stream));
    hipEvent_t e0, e1;
    HIPCHK(s, hipEventCreate(&e0));
    HIPCHK(s, hipEventCreate(&e1));
    // candidates from ncand on (where built): the fused stage pair, timed per stage
    double tbest[24];
    for (double &t : tbest) t = 1e300;
    const double cf[6] = {0.0, 1.0, 0.0, 0.0, 0.0, 0.0};
    for (int pass = 0; pass < 2; ++pass)
        for (int j = 0; j < ncand + npair + nrc; ++j) {
            const bool pair = j >= ncand && j < ncand + npair, recompute = j >= ncand + npair;
            if (pair) {
                s->zchunk2 = s->dim == 3 ? zcp[j - ncand] : 1;
                if (s->dim == 3 && s->zchunk2 > s->nz && j > ncand) continue;
            } else {
                const int k = recompute ? j - ncand - npair : j;
                s->zchunk = s->dim == 3 ? zcs3[k] : 1;
                if (s->dim == 3 && s->zchunk > s->nz && k > 0) continue;
            }
            pf_status rc = PF_OK;
            for (int r = 0; r < 6 && !rc; ++r) {
                if (r == 1) hipEventRecord(e0, s->stream);
                if (pair)
                    rc = stage_pair<T>(s, u, bp<T>(s, w[1]), bp<T>(s, w[2]), bp<T>(s, w[3]), bp<T>(s, w[0]),
                                       bp<T>(s, w[4]), cf, cf);
                else if (recompute)
                    rc = stage<T>(s, K_RKL2_RC, u, bp<T>(s, w[1]), bp<T>(s, w[2]), nullptr, bp<T>(s, w[0]),
                                  nullptr, cf[0], cf[1], cf[2], cf[3], cf[4], cf[5], 0, 1.0);
                else
                    rc = stage<T>(s, K_RKL2, u, bp<T>(s, w[1]), bp<T>(s, w[2]), bp<T>(s, w[3]),
                                  bp<T>(s, w[0]), nullptr, cf[0], cf[1], cf[2], cf[3], cf[4], cf[5], 0);
            }
            if (rc) {
                hipEventDestroy(e0);
                hipEventDestroy(e1);
                return rc;
            }
            HIPCHK(s, hipEventRecord(e1, s->stream));
            HIPCHK(s, hipEventSynchronize(e1));
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            tbest[j] = std::min(tbest[j], ms / (pair ? 10.0 : 5.0));
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    best = 1e300;
    for (int j = 0; j < ncand; ++j)
        if (tbest[j] < best) {
            best = tbest[j];
            bzc = s->dim == 3 ? zcs3[j] : 1;
        }
    fuse = 1;
    r0rc = 0;
    for (int j = ncand + npair; j < ncand + npair + nrc; ++j)
        if (tbest[j] < best) {
            best = tbest[j];
            r0rc = 1;
            bzc = zcs3[j - ncand - npair];
        }
    for (int j = ncand; j < ncand + npair; ++j)
        if (tbest[j] < best) {
            best = tbest[j];
            fuse = 2;
            bzc2 = s->dim == 3 ? zcp[j - ncand] : 1;
        }
    return PF_OK;
}

// Validates a parameter set and fills the host-side description of a
// simulation (no device memory).
pf_status init_meta(pf_sim *s, const pf_params *p) {
    if (p->dim != 2 && p->dim != 3) return PF_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || (p->dim == 2 && p->nz != 1)) return PF_EINVAL;
    if (p->n_phi < 1 || p->n_phi > NMAX || p->n_types < 1 || p->n_types > TMAX) return PF_EINVAL;
    if (!(p->dx > 0) || !(p->W > 0) || !p->type_of || !p->gamma || !p->mob || !p->k || !p->c0 ||
        !p->D)
        return PF_EINVAL;
    if (p->prec != PF_FP64 && p->prec != PF_FP32) return PF_EUNSUPPORTED;
    if (!nphi_supported(p->n_phi)) return PF_EUNSUPPORTED;
    {
        // the kernels address a vector's planes in at most four groups of
        // ceil((N + 1) / groups) planes, each within a 32-bit byte range
        const long long cells = (long long)p->nx * p->ny * p->nz;
        if (field_groups_needed(p->n_phi, cells, p->prec == PF_FP64 ? 8 : 4) == 0)
            return PF_EUNSUPPORTED;
    }
    for (int a = 0; a < p->n_phi; ++a)
        if (p->type_of[a] < 0 || p->type_of[a] >= p->n_types) return PF_EINVAL;
    // pair tables symmetric, finite and non-negative; per-type constants finite
    const int TN = p->n_types;
    for (int i = 0; i < TN; ++i)
        for (int j = 0; j < TN; ++j) {
            const double g = p->gamma[i * TN + j], m = p->mob[i * TN + j];
            if (!std::isfinite(g) || !std::isfinite(m) || g < 0 || m < 0) return PF_EINVAL;
            if (g != p->gamma[j * TN + i] || m != p->mob[j * TN + i]) return PF_EINVAL;
        }
    for (int t = 0; t < TN; ++t)
        if (!(p->k[t] > 0) || !std::isfinite(p->k[t]) || !std::isfinite(p->c0[t]) ||
            !std::isfinite(p->D[t]) || p->D[t] < 0)
            return PF_EINVAL;
    if (p->ssp_stages < 0 || p->ssp_stages == 1) return PF_EINVAL;
    // boundaries: walls per axis, fixed c only on the faces of walled axes
    int walls = 0, cfix = 0;
    for (int a = 0; a < 3; ++a) {
        if (p->bc[a] != 0 && p->bc[a] != 1) return PF_EINVAL;
        if (p->bc[a] == 1) {
            if (a == 2 && p->dim == 2) return PF_EINVAL;
            walls |= 1 << a;
        }
    }
    for (int f = 0; f < 6; ++f)
        if (p->c_fixed[f]) {
            if (!((walls >> (f / 2)) & 1) || !p->with_c || !std::isfinite(p->c_bc[f])) return PF_EINVAL;
            cfix |= 1 << f;
        }
    // wall kernels are built for vectors that fit one buffer group
    if (walls && field_groups_needed(p->n_phi, (long long)p->nx * p->ny * p->nz,
                                     p->prec == PF_FP64 ? 8 : 4) != 1)
        return PF_EUNSUPPORTED;
    s->walls = walls;
    s->cfix = cfix;
    for (int f = 0; f < 6; ++f) s->cbc[f] = (cfix >> f) & 1 ? p->c_bc[f] : 0.0;
    s->dim = p->dim; s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
    s->tx = tile_cols(p->dim);
    s->N = p->n_phi; s->T = p->n_types; s->with_c = p->with_c ? 1 : 0;
    s->ssp_s = p->ssp_stages >= 2 ? p->ssp_stages : 5;
    s->prec = p->prec;
    s->dx = p->dx; s->W = p->W;
    s->type_of.assign(p->type_of, p->type_of + p->n_phi);
    const int TT = p->n_types * p->n_types;
    s->gamma.assign(p->gamma, p->gamma + TT);
    s->mob.assign(p->mob, p->mob + TT);
    s->k.assign(p->k, p->k + p->n_types);
    s->c0.assign(p->c0, p->c0 + p->n_types);
    s->D.assign(p->D, p->D + p->n_types);
    s->F = s->N + s->with_c;
    s->V = (long long)p->nx * p->ny * p->nz;
    s->esz = p->prec == PF_FP64 ? sizeof(double) : sizeof(float);
    return PF_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

pf_status pf_create(const pf_params *p, pf_sim **out) {
    if (!p || !out) return PF_EINVAL;
    *out = nullptr;
    pf_sim *s = new (std::nothrow) pf_sim();
    if (!s) return PF_ENOMEM;
    pf_status rc = init_meta(s, p);
    if (rc) {
        delete s;
        return rc;
    }
    // same result bits either way: pairs by default where they measured faster
    // (2D); in 3D they are an autotuner candidate (latency-bound at two waves
    // per SIMD, slower than single stages on the 512^3 workload)
    s->fuse = pair_ok(s) && s->dim == 2 ? 2 : 1;
    if (p->prec == PF_FP64) {
        DevParams<double> P;
        fill_params(s, P);
        fill_kconsts(P, s->kd);
        if (hipMalloc(&s->dparams, sizeof P) != hipSuccess) rc = PF_ENOMEM;
        else if (hipMemcpy(s->dparams, &P, sizeof P, hipMemcpyHostToDevice) != hipSuccess) rc = PF_EHIP;
    } else {
        DevParams<float> P;
        fill_params(s, P);
        fill_kconsts(P, s->kf);
        if (hipMalloc(&s->dparams, sizeof P) != hipSuccess) rc = PF_ENOMEM;
        else if (hipMemcpy(s->dparams, &P, sizeof P, hipMemcpyHostToDevice) != hipSuccess) rc = PF_EHIP;
    }
    // the reduction kernels write their scalar results straight into this
    // memory, so reading them back needs no copy command
    if (!rc && hipHostMalloc(&s->hres, RES_LEN * sizeof(double),
                             hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        rc = PF_ENOMEM;
    if (!rc) std::memset(s->hres, 0, RES_LEN * sizeof(double));
    if (!rc && hipHostGetDevicePointer((void **)&s->hres_dev, s->hres, 0) != hipSuccess) rc = PF_EHIP;
    if (!rc) rc = ensure_buf(s, 0);
    if (rc) {
        pf_destroy(s);
        return rc;
    }
    *out = s;
    return PF_OK;
}

pf_status pf_destroy(pf_sim *s) {
    if (!s) return PF_EINVAL;
    if (s->stream) hipStreamSynchronize(s->stream);
    else hipDeviceSynchronize();
    for (int i = 0; i < NBUF; ++i)
        if (s->buf[i]) hipFree(s->buf[i]);
    if (s->dparams) hipFree(s->dparams);
    if (s->dcut) hipFree(s->dcut);
    if (s->red) hipFree(s->red);
    if (s->redn) hipFree(s->redn);
    if (s->hres) hipHostFree(s->hres);
    for (auto &p : s->pending) {
        hipEventDestroy(p.e0);
        hipEventDestroy(p.e1);
    }
    for (auto e : s->pool) hipEventDestroy(e);
    delete s;
    return PF_OK;
}

pf_status pf_set_stream(pf_sim *s, void *stream) {
    if (!s) return PF_EINVAL;
    collect_timing(s);
    const hipStream_t next = (hipStream_t)stream;
    // the handle's work queued on the previous stream ends before any of its
    // work on the next one starts (the two streams need not be ordered)
    if (next != s->stream && hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(s, PF_EHIP, "hipStreamSynchronize of the previous stream failed");
    s->stream = next;
    return PF_OK;
}

pf_status pf_init_fields(pf_sim *s, const double *phi, const double *c, double t0) {
    if (!s || !phi) return PF_EINVAL;
    pf_status rc = DISPATCH(s, upload, phi, c);
    if (rc) return rc;
    s->t = t0;
    s->have_fields = true;
    s->ctrl = ctrl_initial();
    s->dt_next = 0.0;
    return PF_OK;
}

pf_status pf_init_fields_device(pf_sim *s, const void *state, double t0) {
    if (!s || !state) return PF_EINVAL;
    if (s->n_p > 0) {
        const hipError_t e = s->prec == PF_FP64
            ? launch_pack_sparse<double>((const double *)state, (double *)s->buf[s->cur], s->N, s->with_c,
                                         s->V, s->n_p, s->ids_off, s->dcut, s->stream)
            : launch_pack_sparse<float>((const float *)state, (float *)s->buf[s->cur], s->N, s->with_c,
                                        s->V, s->n_p, s->ids_off, s->dcut, s->stream);
        if (e != hipSuccess) return fail(s, PF_EHIP, "pack launch: %s", hipGetErrorString(e));
    } else {
        HIPCHK(s, hipMemcpyAsync(s->buf[s->cur], state, state_bytes(s), hipMemcpyDeviceToDevice,
                                 s->stream));
    }
    s->t = t0;
    s->have_fields = true;
    s->ctrl = ctrl_initial();
    s->dt_next = 0.0;
    return PF_OK;
}

pf_status pf_get_fields(pf_sim *s, double *phi, double *c, double *t) {
    if (!s) return PF_EINVAL;
    if (pf_status rc = need_fields(s)) return rc;
    if (t) *t = s->t;
    if (!phi && !c) return PF_OK;
    return DISPATCH(s, download, s->buf[s->cur], phi, c, s->n_p > 0);
}

pf_status pf_get_fields_device(pf_sim *s, void *state) {
    if (!s || !state) return PF_EINVAL;
    if (pf_status rc = need_fields(s)) return rc;
    if (s->n_p > 0) {
        const hipError_t e = s->prec == PF_FP64
            ? launch_unpack_sparse<double>((const double *)s->buf[s->cur], (double *)state, s->N, s->with_c,
                                           s->V, s->n_p, s->ids_off, s->stream)
            : launch_unpack_sparse<float>((const float *)s->buf[s->cur], (float *)state, s->N, s->with_c,
                                          s->V, s->n_p, s->ids_off, s->stream);
        if (e != hipSuccess) return fail(s, PF_EHIP, "unpack launch: %s", hipGetErrorString(e));
        return PF_OK;
    }
    HIPCHK(s, hipMemcpyAsync(state, s->buf[s->cur], state_bytes(s), hipMemcpyDeviceToDevice,
                             s->stream));
    return PF_OK;
}

pf_status pf_rhs_device(pf_sim *s, void *out) {
    if (!s || !out) return PF_EINVAL;
    if (pf_status rc = need_fields(s)) return rc;
    if (s->prec == PF_FP64)
        return stage<double>(s, K_RHS, bp<double>(s, s->cur), nullptr, nullptr, nullptr,
                             (double *)out, nullptr, 0, 0, 0, 0, 0, 0, 0);
    return stage<float>(s, K_RHS, bp<float>(s, s->cur), nullptr, nullptr, nullptr, (float *)out,
                        nullptr, 0, 0, 0, 0, 0, 0, 0);
}

pf_status pf_rhs(pf_sim *s, double *dphi, double *dc) {
    if (!s || !dphi) return PF_EINVAL;
    if (pf_status rc = need_fields(s)) return rc;
    const int w = work_index(s, 0);
    if (pf_status rc = ensure_buf(s, w)) return rc;
    if (pf_status rc = pf_rhs_device(s, s->buf[w])) return rc;
    return DISPATCH(s, download, s->buf[w], dphi, dc);
}

pf_status pf_stable_dt(pf_sim *s, double *dte) {
    if (!s || !dte) return PF_EINVAL;
    *dte = stable_dt(s);
    return PF_OK;
}

pf_status pf_stage_count(pf_sim *s, pf_integrator integ, double dt, int *ns) {
    if (!s || !ns) return PF_EINVAL;
    switch (integ) {
    case PF_FEULER: *ns = 1; return PF_OK;
    case PF_SSP_S2: *ns = s->ssp_s; return PF_OK;
    case PF_SSP_10_4: *ns = 10; return PF_OK;
    case PF_RKL1:
    case PF_RKL2: {
        const int v = stage_count(integ == PF_RKL1 ? 1 : 2, dt, stable_dt(s));
        if (v < 0) return fail(s, PF_EINVAL, "dt must be > 0");
        *ns = v;
        return PF_OK;
    }
    default: return PF_EINVAL;
    }
}

// Sparse phase storage runs forward Euler, RKL1 and RKL2 fixed steps.
static pf_status sparse_integ_ok(pf_sim *s, int integ, const pf_tol *tol) {
    if (s->n_p <= 0) return PF_OK;
    if (tol || (integ != PF_FEULER && integ != PF_RKL1 && integ != PF_RKL2))
        return fail(s, PF_EUNSUPPORTED, "sparse phase storage runs fixed FE, RKL1 and RKL2 steps");
    return PF_OK;
}

pf_status pf_step(pf_sim *s, pf_integrator integ, double dt, pf_stats *stats) {
    if (!s) return PF_EINVAL;
    if (pf_status rc = need_fields(s)) return rc;
    if (pf_status rc = sparse_integ_ok(s, integ, nullptr)) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(s, PF_EINVAL, "dt must be finite and > 0");
    s->st = pf_stats{};
    int ns = s->ssp_s;
    if (integ == PF_RKL1 || integ == PF_RKL2) ns = stage_count(integ == PF_RKL1 ? 1 : 2, dt, stable_dt(s));
    int res, aux;
    pf_status rc = s->prec == PF_FP64 ? do_step<double>(s, integ, ns, dt, false, &res, &aux)
                                      : do_step<float>(s, integ, ns, dt, false, &res, &aux);
    if (rc) return rc;
    s->cur = res;
    s->t += dt;
    s->st.accepted = 1;
    s->st.t = s->t;
    s->st.last_dt = dt;
    if (stats) *stats = s->st;
    return PF_OK;
}

pf_status pf_run_to(pf_sim *s, pf_integrator integ, double t_end, const pf_tol *tol,
                    double dt_fixed, pf_stats *stats) {
    if (!s) return PF_EINVAL;
    if (pf_status rc = need_fields(s)) return rc;
    if (pf_status rc = sparse_integ_ok(s, integ, tol)) return rc;
    if (!std::isfinite(t_end)) return fail(s, PF_EINVAL, "t_end must be finite");
    s->st = pf_stats{};
    pf_status rc = s->prec == PF_FP64 ? run_to_t<double>(s, integ, t_end, tol, dt_fixed)
                                      : run_to_t<float>(s, integ, t_end, tol, dt_fixed);
    s->st.t = s->t;
    if (stats) *stats = s->st;
    return rc;
}

pf_status pf_error_norm_device(pf_sim *s, int kind, double dt, const void *u_old, const void *u_new,
                               const void *aux, const pf_tol *tol, double *norm, long long *ndof) {
    if (!s || !u_old || !u_new || !aux || !tol || !norm) return PF_EINVAL;
    if (s->n_p > 0) return fail(s, PF_EUNSUPPORTED, "error norms need dense storage");
    if (kind != 0 && kind != 1) return PF_EINVAL;
    if (s->prec == PF_FP64)
        return error_norm<double>(s, kind, dt, (const double *)u_old, (const double *)u_new,
                                  (const double *)aux, *tol, norm, ndof);
    return error_norm<float>(s, kind, dt, (const float *)u_old, (const float *)u_new,
                             (const float *)aux, *tol, norm, ndof);
}

pf_status pf_error_norm_device_noalloc(pf_sim *s, int kind, double dt, const void *u_old,
                                       const void *u_new, const void *aux, const pf_tol *tol,
                                       double *norm, long long *ndof) {
    if (!s || !u_old || !u_new || !aux || !tol || !norm) return PF_EINVAL;
    if (kind != 0 && kind != 1) return PF_EINVAL;
    if (s->n_p > 0) return fail(s, PF_EUNSUPPORTED, "error norms need dense storage");
    // the partial sums go to the static scratch: nred doubles, then nred
    // counts from the next 256-byte boundary; every entry is written before
    // the final sum reads it, so nothing needs clearing between calls
    const size_t nred = (size_t)norm_partials(s, kind);
    const size_t cnt_off = (nred * sizeof(double) + 255) / 256 * 256;
    if (cnt_off + nred * sizeof(long long) > SCRATCH_BYTES)
        return fail(s, PF_EINVAL,
                    "%zu partial sums (one per tile of 64 x %d cells and z extent %d) exceed the "
                    "static scratch of %zu bytes (at most %zu); use a larger z extent "
                    "(pf_set_tiling) or pf_error_norm_device",
                    nred, tile_rows(s->dim, s->N), s->dim == 3 ? s->zchunk : 1, (size_t)SCRATCH_BYTES,
                    (size_t)SCRATCH_BYTES / (sizeof(double) + sizeof(long long)));
    void *base = nullptr;
    HIPCHK(s, scratch_address(&base));
    double *red = (double *)base;
    long long *redn = (long long *)((char *)base + cnt_off);
    if (s->prec == PF_FP64)
        return error_norm_with<double>(s, kind, dt, (const double *)u_old, (const double *)u_new,
                                       (const double *)aux, *tol, red, redn, false, norm, ndof);
    return error_norm_with<float>(s, kind, dt, (const float *)u_old, (const float *)u_new,
                                  (const float *)aux, *tol, red, redn, false, norm, ndof);
}

pf_status pf_error_norm(const pf_params *p, long long cells, const double *e, const double *u_old,
                        const double *u_new, const pf_tol *tol, double *out) {
    if (!p || !e || !u_old || !u_new || !tol || !out || cells < 1) return PF_EINVAL;
    if (p->n_phi < 1 || p->n_phi > NMAX) return PF_EINVAL;
    if (!(tol->r_phi >= 0.0) || !(tol->a_phi >= 0.0) || !(tol->r_c >= 0.0) || !(tol->a_c >= 0.0))
        return PF_EINVAL;
    const int N = p->n_phi;
    const long long V = cells;
    // eq. error_norm: cells in order; in each cell the phi entries with a
    // nonzero estimate (phases ascending), or two degrees of freedom where
    // there are none, then the cell's c entry
    double sum = 0.0;
    long long ndof = 0;
    for (long long i = 0; i < V; ++i) {
        int nt = 0;
        for (int a = 0; a < N; ++a) {
            const long long k = (long long)a * V + i;
            if (e[k] != 0.0) {
                const double w = tol->r_phi * std::fmax(std::fabs(u_old[k]), std::fabs(u_new[k])) + tol->a_phi;
                const double q = e[k] / w;
                sum = sum + q * q;
                ++nt;
            }
        }
        ndof += nt > 0 ? nt : 2;
        if (p->with_c) {
            const long long k = (long long)N * V + i;
            const double w = tol->r_c * std::fmax(std::fabs(u_old[k]), std::fabs(u_new[k])) + tol->a_c;
            const double q = e[k] / w;
            sum = sum + q * q;
            ndof += 1;
        }
    }
    *out = std::sqrt(sum / (double)ndof);
    return PF_OK;
}

pf_status pf_set_field_groups(pf_sim *s, int ng) {
    if (!s) return PF_EINVAL;
    if (ng != 0 && ng != 1 && ng != 2 && ng != 4)
        return fail(s, PF_EINVAL, "buffer groups %d (0, 1, 2 or 4)", ng);
    const int need = field_groups_needed(s->N, s->V, (int)s->esz);
    if (ng != 0 && ng < need)
        return fail(s, PF_EINVAL, "the vectors need at least %d buffer groups", need);
    if (ng > 1 && s->walls)
        return fail(s, PF_EUNSUPPORTED, "wall kernels are built for one buffer group");
    s->groups_min = ng == 0 ? 1 : ng;
    return PF_OK;
}

pf_status pf_get_field_groups(const pf_sim *s, int *ng) {
    if (!s || !ng) return PF_EINVAL;
    *ng = sim_groups(s);
    return PF_OK;
}

pf_status pf_set_sparse_storage(pf_sim *s, int n_p) {
    if (!s) return PF_EINVAL;
    if (n_p < 0 || n_p > SPMAX || n_p > s->N)
        return fail(s, PF_EINVAL, "n_p = %d (0 for dense, else 1..%d and at most N)", n_p, SPMAX);
    if (n_p > 0) {
        if (s->walls) return fail(s, PF_EUNSUPPORTED, "sparse phase storage needs periodic grids");
        int ng = std::max(std::max(field_groups_needed(s->N, s->V, (int)s->esz),
                                   field_groups_needed(SPMAX, s->V, (int)s->esz)), s->groups_min);
        if (ng == 0 || ng > 2)
            return fail(s, PF_EUNSUPPORTED, "sparse phase storage is built for one or two buffer groups");
    }
    if (s->stream) hipStreamSynchronize(s->stream);
    else hipDeviceSynchronize();
    for (int i = 0; i < NBUF; ++i)
        if (s->buf[i]) {
            hipFree(s->buf[i]);
            s->buf[i] = nullptr;
        }
    s->cur = 0;
    s->have_fields = false;
    s->n_p = n_p;
    s->ids_off = n_p > 0 ? ((unsigned long long)(n_p + 1) * (unsigned long long)s->V * s->esz + 255) / 256 * 256 : 0;
    if (n_p > 0 && !s->dcut) {
        if (hipMalloc(&s->dcut, sizeof(unsigned long long)) != hipSuccess) {
            s->dcut = nullptr;
            s->n_p = 0;
            s->ids_off = 0;
            return fail(s, PF_ENOMEM, "cut counter");
        }
    }
    if (s->dcut) HIPCHK(s, hipMemset(s->dcut, 0, sizeof(unsigned long long)));
    s->fuse = pair_ok(s) && s->dim == 2 ? 2 : 1;
    return ensure_buf(s, 0);
}

pf_status pf_get_sparse_storage(const pf_sim *s, int *n_p) {
    if (!s || !n_p) return PF_EINVAL;
    *n_p = s->n_p;
    return PF_OK;
}

pf_status pf_sparse_cuts(pf_sim *s, long long *cuts) {
    if (!s || !cuts) return PF_EINVAL;
    *cuts = 0;
    if (!s->dcut) return PF_OK;
    unsigned long long v = 0;
    HIPCHK(s, hipMemcpyAsync(&v, s->dcut, sizeof v, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    HIPCHK(s, hipMemsetAsync(s->dcut, 0, sizeof v, s->stream));
    *cuts = (long long)v;
    return PF_OK;
}

}  // extern "C"

namespace {
// The diagnostics reduction over the current state; phases == false reads c
// only (the sum of c is formed in the same order either way, so it has the
// same bits).
pf_status diag_run(pf_sim *s, bool phases, double out[5]) {
    if (pf_status rc = need_fields(s)) return rc;
    const int nb = 1024;
    if (pf_status rc = ensure_red(s, nb)) return rc;
    Pending p;
    begin_timed(s, FAM_RED, p);
    // dense: N phase planes then c; sparse: c, then n_p slots (empty ones 0)
    const bool sp = s->n_p > 0;
    const int nphi = !phases ? 0 : sp ? s->n_p : s->N;
    const long long po = sp ? s->V : 0, co = sp ? 0 : (long long)s->N * s->V;
    hipError_t e = s->prec == PF_FP64
                       ? launch_diag<double>((const double *)s->buf[s->cur] + po,
                                             (const double *)s->buf[s->cur] + co, nphi, s->with_c,
                                             s->V, s->red, nb, s->stream)
                       : launch_diag<float>((const float *)s->buf[s->cur] + po,
                                            (const float *)s->buf[s->cur] + co, nphi, s->with_c, s->V,
                                            s->red, nb, s->stream);
    if (e != hipSuccess) return fail(s, PF_EHIP, "diag launch: %s", hipGetErrorString(e));
    HIPCHK(s, launch_finalize_diag(s->red, nb, s->hres_dev + RES_DIAG, s->stream));
    end_timed(s, p);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int k = 0; k < 5; ++k) out[k] = s->hres[RES_DIAG + k];
    return PF_OK;
}
}  // namespace

extern "C" {

pf_status pf_diagnostics(pf_sim *s, double out[5]) {
    if (!s || !out) return PF_EINVAL;
    return diag_run(s, true, out);
}

pf_status pf_conservation(pf_sim *s, double *sum_c) {
    if (!s || !sum_c) return PF_EINVAL;
    double d[5];
    pf_status rc = diag_run(s, false, d);
    if (rc) return rc;
    *sum_c = d[0];
    return PF_OK;
}

pf_status pf_get_trace(pf_sim *s, double *buf, long long cap, long long *n) {
    if (!s || !n) return PF_EINVAL;
    const long long rows = (long long)s->trace.size() / 4;
    *n = rows;
    if (buf && cap > 0)
        std::memcpy(buf, s->trace.data(), sizeof(double) * 4 * (size_t)std::min(rows, cap));
    return PF_OK;
}

pf_status pf_get_state(pf_sim *s, void *buf, size_t *len) {
    if (!s || !len) return PF_EINVAL;
    if (s->n_p > 0) return fail(s, PF_EUNSUPPORTED, "checkpoints need dense storage");
    if (pf_status rc = need_fields(s)) return rc;
    const size_t need = sizeof(CkptHeader) + state_bytes(s);
    if (!buf) {
        *len = need;
        return PF_OK;
    }
    if (*len < need) return fail(s, PF_EINVAL, "buffer too small (%zu < %zu)", *len, need);
    CkptHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "PFCKPT1", 8);
    h.prec = s->prec; h.F = s->F; h.V = s->V; h.t = s->t; h.dt_next = s->dt_next;
    h.b = s->ctrl.b; h.E1 = s->ctrl.E1; h.E2 = s->ctrl.E2; h.h1 = s->ctrl.h1; h.h2 = s->ctrl.h2;
    h.nhist = s->ctrl.nhist; h.st = s->st;
    std::memcpy(buf, &h, sizeof h);
    HIPCHK(s, hipMemcpyAsync((char *)buf + sizeof h, s->buf[s->cur], state_bytes(s),
                             hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *len = need;
    return PF_OK;
}

pf_status pf_set_state(pf_sim *s, const void *buf, size_t len) {
    if (!s || !buf) return PF_EINVAL;
    if (s->n_p > 0) return fail(s, PF_EUNSUPPORTED, "checkpoints need dense storage");
    CkptHeader h;
    if (len < sizeof h) return fail(s, PF_EINVAL, "checkpoint too short");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, "PFCKPT1", 8) != 0 || h.prec != s->prec || h.F != s->F || h.V != s->V ||
        len < sizeof h + state_bytes(s))
        return fail(s, PF_EINVAL, "checkpoint does not match this handle");
    HIPCHK(s, hipMemcpyAsync(s->buf[s->cur], (const char *)buf + sizeof h, state_bytes(s),
                             hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->t = h.t; s->dt_next = h.dt_next;
    s->ctrl.b = h.b; s->ctrl.E1 = h.E1; s->ctrl.E2 = h.E2; s->ctrl.h1 = h.h1; s->ctrl.h2 = h.h2;
    s->ctrl.nhist = h.nhist; s->st = h.st;
    s->have_fields = true;
    return PF_OK;
}

pf_status pf_set_tiling(pf_sim *s, int tx, int zchunk) {
    if (!s) return PF_EINVAL;
    if (tx != 0 && tx != tile_cols(s->dim))
        return fail(s, PF_EINVAL, "tx must be 0 or %d (the tile width of %dD grids)", tile_cols(s->dim),
                    s->dim);
    if (zchunk < 1) return fail(s, PF_EINVAL, "zchunk must be >= 1");
    s->zchunk = zchunk;
    return PF_OK;
}

pf_status pf_get_tiling(pf_sim *s, int *tx, int *zchunk) {
    if (!s || !tx || !zchunk) return PF_EINVAL;
    *tx = s->tx;
    *zchunk = s->zchunk;
    return PF_OK;
}

pf_status pf_autotune(pf_sim *s, int *tx_out, int *zc_out, double *best_ms) {
    if (!s) return PF_EINVAL;
    if (pf_status rc = need_fields(s)) return rc;
    int w[5] = {-1, -1, -1, -1, -1};
    for (int k = 0; k < (pair_ok(s) ? 5 : 4); ++k) {
        w[k] = work_index(s, k);
        if (pf_status rc = ensure_buf(s, w[k])) return rc;
    }
    const bool was_timing = s->timing;
    s->timing = false;
    double best;
    int bzc = s->zchunk, fuse = 1, bzc2 = s->zchunk2, r0rc = 0;
    pf_status rc = s->prec == PF_FP64 ? autotune_t<double>(s, w, best, bzc, fuse, bzc2, r0rc)
                                      : autotune_t<float>(s, w, best, bzc, fuse, bzc2, r0rc);
    s->timing = was_timing;
    if (rc) return rc;
    s->zchunk = bzc;
    s->zchunk2 = bzc2;
    s->fuse = fuse;
    s->r0rc = r0rc;
    if (tx_out) *tx_out = s->tx;
    if (zc_out) *zc_out = bzc;
    if (best_ms) *best_ms = best;
    return PF_OK;
}

pf_status pf_set_stage_fusion(pf_sim *s, int depth) {
    if (!s) return PF_EINVAL;
    if (depth != 1 && depth != 2) return fail(s, PF_EINVAL, "stage fusion depth %d (1 or 2)", depth);
    if (depth == 2 && !pair_ok(s))
        return fail(s, PF_EUNSUPPORTED, "fused RKL2 stage pairs are built for periodic grids: in 2D "
                                        "where the vectors fit one buffer group and the LDS fits, "
                                        "in 3D for single precision with N <= %d and double "
                                        "precision with N <= %d", P3_NMAX32, P3_NMAX64);
    s->fuse = depth;
    return PF_OK;
}

pf_status pf_set_r0_recompute(pf_sim *s, int on) {
    if (!s) return PF_EINVAL;
    if (on != 0 && on != 1) return fail(s, PF_EINVAL, "r0 recompute %d (0 or 1)", on);
    if (on && !rc_ok(s))
        return fail(s, PF_EUNSUPPORTED, "RKL2 stages that recompute R0 are built for periodic 3D grids "
                                        "in dense storage, single precision N <= 9, double N <= 4");
    s->r0rc = on;
    return PF_OK;
}

pf_status pf_get_r0_recompute(const pf_sim *s, int *on) {
    if (!s || !on) return PF_EINVAL;
    *on = s->r0rc;
    return PF_OK;
}

pf_status pf_get_stage_fusion(const pf_sim *s, int *depth) {
    if (!s || !depth) return PF_EINVAL;
    *depth = s->fuse;
    return PF_OK;
}

pf_status pf_set_pair_zchunk(pf_sim *s, int zchunk) {
    if (!s) return PF_EINVAL;
    if (zchunk < 1) return fail(s, PF_EINVAL, "zchunk must be >= 1");
    s->zchunk2 = zchunk;
    return PF_OK;
}

pf_status pf_get_pair_zchunk(const pf_sim *s, int *zchunk) {
    if (!s || !zchunk) return PF_EINVAL;
    *zchunk = s->zchunk2;
    return PF_OK;
}

pf_status pf_set_timing_families(pf_sim *s, unsigned families) {
    if (!s) return PF_EINVAL;
    collect_timing(s);
    s->timing = families != 0;
    s->timing_mask = families & 31u;
    for (int f = 0; f < 5; ++f) {
        s->fam_ms[f] = 0.0;
        s->fam_n[f] = 0;
    }
    return PF_OK;
}

pf_status pf_set_timing(pf_sim *s, int enable) {
    return pf_set_timing_families(s, enable ? 31u : 0u);
}

pf_status pf_get_kernel_time(pf_sim *s, int family, double *ms, long long *launches) {
    if (!s || family < 0 || family > 4 || !ms) return PF_EINVAL;
    collect_timing(s);
    *ms = s->fam_ms[family];
    if (launches) *launches = s->fam_n[family];
    return PF_OK;
}

int pf_supported_nphi(int *out, int cap) { return supported_nphi_list(out, cap); }

pf_status pf_params_stable_dt(const pf_params *p, double *dt_e) {
    if (!p || !dt_e) return PF_EINVAL;
    pf_sim meta;
    if (pf_status rc = init_meta(&meta, p)) return rc;
    *dt_e = stable_dt(&meta);
    return PF_OK;
}

pf_status pf_rkl_stage_count(pf_integrator integ, double dt, double dt_e, int *ns) {
    if (!ns || (integ != PF_RKL1 && integ != PF_RKL2)) return PF_EINVAL;
    const int v = stage_count(integ == PF_RKL1 ? 1 : 2, dt, dt_e);
    if (v < 0) return PF_EINVAL;
    *ns = v;
    return PF_OK;
}

pf_status pf_controller_init(pf_controller *c) {
    if (!c) return PF_EINVAL;
    *c = ctrl_initial();
    return PF_OK;
}

pf_status pf_controller_update(pf_controller *c, int order, double err, double h, int *accept,
                               double *h_next) {
    if (!c || !accept || !h_next || order < 1 || !(h > 0.0)) return PF_EINVAL;
    bool acc = false;
    *h_next = ctrl_update(*c, order, err, h, acc);
    *accept = acc ? 1 : 0;
    return PF_OK;
}

int pf_clip_step(double t, double t_end, double h, double *h_use, int *last) {
    if (!h_use || !last || !(h > 0.0)) return -1;
    bool l = false;
    double hu = 0.0;
    if (!clip_step(t, t_end, h, hu, l)) return 0;
    *h_use = hu;
    *last = l ? 1 : 0;
    return 1;
}

const char *pf_last_error(const pf_sim *s) { return s ? s->err.c_str() : "null handle"; }

}  // extern "C"

// ===========================================================================
// Batch of independent 2D simulations (one fused launch per step for all)
// ===========================================================================

struct pf_batch {
    int n = 0, N = 0, F = 0, with_c = 0;
    pf_precision prec = PF_FP32;
    size_t esz = 4;
    std::vector<pf_sim> meta;      // per-instance parameters (no device memory)
    std::vector<long long> off;    // element offsets in the batch buffers
    long long total = 0;           // elements per batch buffer
    std::vector<int> ntx, nty, tile0;
    int total_tiles = 0;
    void *bufA = nullptr, *bufB = nullptr;
    // RKL2 runs: ring slots (bufB is the first), the slot-0 store and R0,
    // allocated on the first RKL2 run; the stage coefficient table
    void *bufQ2 = nullptr, *bufS0 = nullptr, *bufR0 = nullptr;
    void *dcoef = nullptr;
    size_t coef_bytes = 0;
    int coef_stride = 0;  // stages + 1 of the longest step
    int integ = PF_FEULER;  // integrator of the current run
    void *dparams = nullptr, *dinst = nullptr;
    int *dtile = nullptr, *dstep = nullptr;
    std::vector<double> t;
    std::vector<int> have;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int nblocks = 2048;
    int depth = 1;                 // steps per batched launch (stage-fusion depth)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_k = 0, graph_depth = 0, graph_blocks = 0, graph_integ = -1, graph_stages = 0;
    // adaptive runs (allocated on the first): the new state, per-tile error
    // partials, per-instance control words (tile0, tiles, active, accepted),
    // state offsets and lengths, norms, and the host-visible copy of the norms
    // followed by their sequence number
    void *bufY = nullptr;
    double *dred = nullptr, *dnorm = nullptr;
    long long *dredn = nullptr, *dlen = nullptr;
    int *dctl = nullptr;
    double *hnorm = nullptr, *hnorm_dev = nullptr;
    double norm_seq = 0.0;
    std::string err;
};

namespace {

pf_status bfail(pf_batch *b, pf_status code, const char *fmt, ...) {
    if (b) {
        char m[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(m, sizeof m, fmt, ap);
        va_end(ap);
        b->err = m;
    }
    return code;
}

#define BHIPCHK(b, expr)                                                                \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return bfail((b), PF_EHIP, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

template <typename T>
BatchArgs<T> batch_args(pf_batch *b, int offset, int depth) {
    BatchArgs<T> B;
    B.params = (const DevParams<T> *)b->dparams;
    B.inst = (const BatchInst<T> *)b->dinst;
    B.tile_inst = b->dtile;
    B.bufA = (T *)b->bufA;
    B.bufB = (T *)b->bufB;
    B.step_base = b->dstep;
    B.step_offset = offset;
    B.total_tiles = b->total_tiles;
    B.depth = depth;
    B.kind = K_EULER;
    B.stage = 0;
    for (int v = 0; v < 6; ++v) B.role[v] = nullptr;
    B.state = (T *)b->bufA;
    B.coef = (const T *)b->dcoef;
    B.coef_stride = b->coef_stride;
    return B;
}

// Arguments of stage j (1..) of an RKL2 step of the batch (step offset k): the
// buffer roles of the single-instance scheme (u^{n,0} = state A, R0, and the
// ring of three stage slots whose slot 0 is u^{n,0} until stage 3 overwrites
// it from a store of its own).
template <typename T>
BatchArgs<T> batch_rkl2_args(pf_batch *b, int k, int j) {
    BatchArgs<T> B = batch_args<T>(b, k, 1);
    T *U = (T *)b->bufA, *W0 = (T *)b->bufB, *W1 = (T *)b->bufQ2, *S0 = (T *)b->bufS0,
      *R0 = (T *)b->bufR0;
    B.stage = j;
    if (j == 1) {
        B.kind = K_RKL2_FIRST;
        B.role[0] = U;
        B.role[4] = W0;
        B.role[5] = R0;
        return B;
    }
    T *slot[3] = {j >= 3 ? S0 : U, W0, W1};
    B.kind = K_RKL2;
    B.role[0] = slot[(j - 1) % 3];
    B.role[1] = slot[(j - 2) % 3];
    B.role[2] = U;
    B.role[3] = R0;
    B.role[4] = slot[j % 3];
    return B;
}

bool batch_depth_ok(const pf_batch *b, int depth) {
    return depth == 1 || (depth == 2 && batch_depth2_fits((int)b->esz, b->N));
}

template <typename T>
pf_status batch_setup_params(pf_batch *b) {
    std::vector<DevParams<T>> P(b->n);
    for (int i = 0; i < b->n; ++i) fill_params(&b->meta[i], P[i]);
    BHIPCHK(b, hipMalloc(&b->dparams, sizeof(DevParams<T>) * b->n));
    BHIPCHK(b, hipMemcpy(b->dparams, P.data(), sizeof(DevParams<T>) * b->n, hipMemcpyHostToDevice));
    BHIPCHK(b, hipMalloc(&b->dinst, sizeof(BatchInst<T>) * b->n));
    return PF_OK;
}

// Step sizes of each instance for a run to t_end[i]: the same clipping rule as
// pf_run_to (full steps of dt, the last one landing on t_end), so every
// instance takes bit for bit the steps a single-instance run would take.
template <typename T>
pf_status batch_plan(pf_batch *b, const double *t_end, const double *dt, int &max_steps,
                     int &max_stages) {
    std::vector<BatchInst<T>> I(b->n);
    std::vector<double> hfull(b->n), hclip(b->n);  // step sizes in double
    max_steps = 0;
    max_stages = 1;
    const bool rkl2 = b->integ == PF_RKL2;
    for (int i = 0; i < b->n; ++i) {
        const double dte = stable_dt(&b->meta[i]);
        const double h0 = dt ? dt[i] : 0.9 * dte;
        if (!(h0 > 0.0)) return bfail(b, PF_EINVAL, "instance %d: dt must be > 0", i);
        double t = b->t[i];
        long long nst = 0;
        double hlast = h0;
        bool clipped = false;
        for (;;) {
            double h;
            bool last;
            if (!clip_step(t, t_end[i], h0, h, last)) break;
            ++nst;
            if (nst > 100000000) return bfail(b, PF_EINVAL, "instance %d: too many steps", i);
            if (last) {
                hlast = h;
                clipped = true;
            }
            t = last ? t_end[i] : t + h;
        }
        I[i].off = b->off[i];
        I[i].ntx = b->ntx[i];
        I[i].nty = b->nty[i];
        I[i].tile0 = b->tile0[i];
        I[i].nsteps = (int)nst;
        I[i].nfull = (int)(clipped ? nst - 1 : nst);
        I[i].dt = (T)h0;
        I[i].dt_last = (T)hlast;
        hfull[i] = h0;
        hclip[i] = hlast;
        I[i].s_full = rkl2 ? stage_count(2, h0, dte) : 1;
        I[i].s_last = rkl2 ? stage_count(2, hlast, dte) : 1;
        if (I[i].s_full < 0 || I[i].s_last < 0) return bfail(b, PF_EINVAL, "instance %d: bad dt", i);
        max_steps = std::max(max_steps, (int)nst);
        if (nst > 0) max_stages = std::max(max_stages, std::max(I[i].s_full, I[i].s_last));
    }
    if (rkl2) {
        // coefficients exactly as the single-instance step passes them
        b->coef_stride = max_stages + 1;
        std::vector<T> cf((size_t)b->n * 2 * b->coef_stride * 6, T(0));
        for (int i = 0; i < b->n; ++i)
            for (int c = 0; c < 2; ++c) {
                const int ns = c ? I[i].s_last : I[i].s_full;
                const double hd = c ? hclip[i] : hfull[i];
                for (int j = 1; j <= ns; ++j) {
                    double mu, nu, mut, gam;
                    rkl_coeffs(2, ns, j, mu, nu, mut, gam);
                    T *e = &cf[((size_t)(2 * i + c) * b->coef_stride + j) * 6];
                    if (j == 1) {
                        e[0] = (T)(mut * hd);
                    } else {
                        e[0] = (T)((1.0 - mu) - nu);
                        e[1] = (T)mu;
                        e[2] = (T)nu;
                        e[3] = (T)hd;
                        e[4] = (T)mut;
                        e[5] = (T)gam;
                    }
                }
            }
        const size_t bytes = cf.size() * sizeof(T);
        if (bytes > b->coef_bytes) {
            if (b->dcoef) hipFree(b->dcoef);
            b->dcoef = nullptr;
            b->coef_bytes = 0;
            BHIPCHK(b, hipMalloc(&b->dcoef, bytes));
            b->coef_bytes = bytes;
        }
        BHIPCHK(b, hipMemcpyAsync(b->dcoef, cf.data(), bytes, hipMemcpyHostToDevice, b->stream));
        BHIPCHK(b, hipStreamSynchronize(b->stream));  // cf is a local
    }
    BHIPCHK(b, hipMemcpyAsync(b->dinst, I.data(), sizeof(BatchInst<T>) * b->n, hipMemcpyHostToDevice,
                              b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));  // I is a local
    return PF_OK;
}

// k batched launches (forward Euler: b->depth steps each, launch j covering the
// steps from the device counter + j * depth on; RKL2: one step of `stages`
// stage launches each) and one counter update by the steps taken.
template <typename T>
pf_status batch_launch_steps(pf_batch *b, int k, int stages) {
    const int d = b->integ == PF_RKL2 ? 1 : b->depth;
    for (int j = 0; j < k; ++j) {
        hipError_t e = hipSuccess;
        if (b->integ == PF_RKL2) {
            for (int st = 1; st <= stages && e == hipSuccess; ++st)
                e = launch_batch_euler<T>(b->N, batch_rkl2_args<T>(b, j, st), b->nblocks, b->stream);
        } else {
            e = launch_batch_euler<T>(b->N, batch_args<T>(b, j * d, d), b->nblocks, b->stream);
        }
        if (e != hipSuccess) return bfail(b, PF_EHIP, "batch launch: %s", hipGetErrorString(e));
    }
    BHIPCHK(b, launch_batch_tick(b->dstep, k * d, b->stream));
    return PF_OK;
}

// k launches (and one counter update) captured once into a hipGraph and
// replayed; the graph holds kernel nodes only.  A change of k, of the fusion
// depth, of the grid size, of the integrator or of the stage count re-captures
// it (the buffers and the coefficient table it refers to stay allocated).
template <typename T>
pf_status batch_graph(pf_batch *b, int k, int stages) {
    if (b->gexec && b->graph_k == k && b->graph_depth == b->depth && b->graph_blocks == b->nblocks &&
        b->graph_integ == b->integ && b->graph_stages == stages)
        return PF_OK;
    if (b->gexec) {
        hipGraphExecDestroy(b->gexec);
        hipGraphDestroy(b->graph);
        b->gexec = nullptr;
        b->graph = nullptr;
    }
    BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    pf_status rc = batch_launch_steps<T>(b, k, stages);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bfail(b, PF_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return bfail(b, PF_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    b->graph = g;
    b->graph_k = k;
    b->graph_depth = b->depth;
    b->graph_blocks = b->nblocks;
    b->graph_integ = b->integ;
    b->graph_stages = stages;
    return PF_OK;
}

template <typename T>
pf_status batch_rkl2_buffers(pf_batch *b) {
    void **bufs[3] = {&b->bufQ2, &b->bufS0, &b->bufR0};
    for (void **q : bufs)
        if (!*q) {
            if (hipMalloc(q, b->total * b->esz) != hipSuccess) {
                *q = nullptr;
                return bfail(b, PF_ENOMEM, "batch RKL2 buffers");
            }
            BHIPCHK(b, hipMemset(*q, 0, b->total * b->esz));
        }
    return PF_OK;
}

template <typename T>
pf_status batch_adaptive_buffers(pf_batch *b) {
    if (b->hnorm) return PF_OK;
    const int n = b->n;
    if (hipMalloc(&b->bufY, b->total * b->esz) != hipSuccess ||
        hipMalloc((void **)&b->dred, sizeof(double) * b->total_tiles) != hipSuccess ||
        hipMalloc((void **)&b->dredn, sizeof(long long) * b->total_tiles) != hipSuccess ||
        hipMalloc((void **)&b->dnorm, sizeof(double) * 3 * n) != hipSuccess ||
        hipMalloc((void **)&b->dctl, sizeof(int) * 4 * n) != hipSuccess ||
        hipMalloc((void **)&b->dlen, sizeof(long long) * 2 * n) != hipSuccess)
        return bfail(b, PF_ENOMEM, "batch adaptive buffers");
    BHIPCHK(b, hipMemset(b->bufY, 0, b->total * b->esz));
    std::vector<long long> ol(2 * n);
    for (int i = 0; i < n; ++i) {
        ol[i] = b->off[i];
        ol[n + i] = (long long)b->meta[i].F * b->meta[i].V;
    }
    BHIPCHK(b, hipMemcpy(b->dlen, ol.data(), sizeof(long long) * 2 * n, hipMemcpyHostToDevice));
    void *h = nullptr;
    if (hipHostMalloc(&h, sizeof(double) * (3 * n + 1), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return bfail(b, PF_ENOMEM, "batch norm buffer");
    b->hnorm = (double *)h;
    for (int k = 0; k <= 3 * n; ++k) b->hnorm[k] = 0.0;
    BHIPCHK(b, hipHostGetDevicePointer((void **)&b->hnorm_dev, h, 0));
    return PF_OK;
}

// Polls the host-visible norm buffer for sequence number seq (see wait_result).
pf_status batch_wait_norms(pf_batch *b, double seq) {
    volatile const double *flag = b->hnorm + 3 * b->n;
    for (unsigned long it = 1;; ++it) {
        if (*flag == seq) break;
        if ((it & 4095u) == 0) {
            const hipError_t q = hipStreamQuery(b->stream);
            if (q == hipSuccess) {
                if (*flag == seq) break;
                return bfail(b, PF_EHIP, "norm results missing after the stream drained");
            }
            if (q != hipErrorNotReady) return bfail(b, PF_EHIP, "stream: %s", hipGetErrorString(q));
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return PF_OK;
}

// Adaptive RKL2 steps of every instance to its t_end (Sec. 3.3): each instance
// runs the single-instance adaptive loop of run_to_t with its own controller,
// step and stage count.  One batch step launches the stages of all instances
// still running (each with its own coefficients; the last stage writes the new
// state into bufY), the estimate, the per-instance norms and their copy to the
// host; the host updates every controller, and a copy kernel moves the new
// state of the accepted instances into the state buffer.  A rejected instance
// keeps its state and retries with the controller's smaller step.
template <typename T>
pf_status batch_run_adaptive(pf_batch *b, const double *t_end, const pf_tol &tol, pf_stats *stats) {
    pf_status rc;
    if ((rc = batch_rkl2_buffers<T>(b)) || (rc = batch_adaptive_buffers<T>(b))) return rc;
    if (b->gexec) {  // the coefficient table may move; a cached graph would refer to it
        hipGraphExecDestroy(b->gexec);
        hipGraphDestroy(b->graph);
        b->gexec = nullptr;
        b->graph = nullptr;
    }
    const int n = b->n;
    const double ratio = tol.dt_max_over_dte > 0.0 ? tol.dt_max_over_dte : 200.0;
    std::vector<double> dte(n), dt(n), h(n);
    std::vector<pf_controller> ctrl(n, ctrl_initial());
    std::vector<pf_stats> st(n, pf_stats{});
    std::vector<int> nonfinite(n, 0), done(n, 0), ns(n, 0), ctl(4 * n);
    std::vector<char> last(n, 0);
    std::vector<BatchInst<T>> I(n);
    std::vector<T> cf;
    long long max_len = 1;
    for (int i = 0; i < n; ++i) {
        dte[i] = stable_dt(&b->meta[i]);
        dt[i] = tol.dt0 > 0.0 ? tol.dt0 : 0.9 * dte[i];
        max_len = std::max(max_len, (long long)b->meta[i].F * b->meta[i].V);
    }
    const int zero = 0;
    BHIPCHK(b, hipMemcpyAsync(b->dstep, &zero, sizeof(int), hipMemcpyHostToDevice, b->stream));
    pf_status fail_rc = PF_OK;
    while (!fail_rc) {
        int active = 0, max_s = 1;
        for (int i = 0; i < n; ++i) {
            BatchInst<T> &q = I[i];
            q = BatchInst<T>{};
            q.off = b->off[i];
            q.ntx = b->ntx[i];
            q.nty = b->nty[i];
            q.tile0 = b->tile0[i];
            ctl[4 * i] = b->tile0[i];
            ctl[4 * i + 1] = b->ntx[i] * b->nty[i];
            ctl[4 * i + 2] = ctl[4 * i + 3] = 0;
            if (done[i]) continue;
            bool li;
            if (!clip_step(b->t[i], t_end[i], std::min(dt[i], ratio * dte[i]), h[i], li)) {
                done[i] = 1;
                continue;
            }
            if (!li && std::isfinite(dte[i]) && h[i] < 1e-12 * dte[i])
                return bfail(b, PF_EDTMIN, "instance %d: adaptive step underflow (dt = %g)", i, h[i]);
            last[i] = li;
            ns[i] = stage_count(2, h[i], dte[i]);
            if (ns[i] < 1) return bfail(b, PF_EINVAL, "instance %d: bad step %g", i, h[i]);
            q.nsteps = q.nfull = 1;
            q.s_full = q.s_last = ns[i];
            q.dt = q.dt_last = (T)h[i];
            q.dt6 = (T)(6.0 * h[i]);
            q.hdt = (T)(h[i] / 2.0);
            ctl[4 * i + 2] = 1;
            ++active;
            max_s = std::max(max_s, ns[i]);
        }
        if (!active) break;
        // coefficients of every running instance's step, as the single-instance
        // step passes them (row 2 i: a full step)
        b->coef_stride = max_s + 1;
        cf.assign((size_t)n * 2 * b->coef_stride * 6, T(0));
        for (int i = 0; i < n; ++i) {
            if (!ctl[4 * i + 2]) continue;
            for (int j = 1; j <= ns[i]; ++j) {
                double mu, nu, mut, gam;
                rkl_coeffs(2, ns[i], j, mu, nu, mut, gam);
                T *e = &cf[((size_t)(2 * i) * b->coef_stride + j) * 6];
                if (j == 1) {
                    e[0] = (T)(mut * h[i]);
                } else {
                    e[0] = (T)((1.0 - mu) - nu);
                    e[1] = (T)mu;
                    e[2] = (T)nu;
                    e[3] = (T)h[i];
                    e[4] = (T)mut;
                    e[5] = (T)gam;
                }
            }
        }
        const size_t bytes = cf.size() * sizeof(T);
        if (bytes > b->coef_bytes) {
            BHIPCHK(b, hipStreamSynchronize(b->stream));
            if (b->dcoef) hipFree(b->dcoef);
            b->dcoef = nullptr;
            b->coef_bytes = 0;
            BHIPCHK(b, hipMalloc(&b->dcoef, bytes));
            b->coef_bytes = bytes;
        }
        BHIPCHK(b, hipMemcpyAsync(b->dcoef, cf.data(), bytes, hipMemcpyHostToDevice, b->stream));
        BHIPCHK(b, hipMemcpyAsync(b->dinst, I.data(), sizeof(BatchInst<T>) * n, hipMemcpyHostToDevice,
                                  b->stream));
        BHIPCHK(b, hipMemcpyAsync(b->dctl, ctl.data(), sizeof(int) * 4 * n, hipMemcpyHostToDevice,
                                  b->stream));
        hipError_t e = hipSuccess;
        for (int j = 1; j <= max_s && e == hipSuccess; ++j) {
            BatchArgs<T> B = batch_rkl2_args<T>(b, 0, j);
            B.state = (T *)b->bufY;
            e = launch_batch_euler<T>(b->N, B, b->nblocks, b->stream);
        }
        if (e == hipSuccess) {
            BatchArgs<T> B = batch_args<T>(b, 0, 1);
            B.kind = K_EST;
            B.role[0] = (const T *)b->bufY;
            B.role[2] = (const T *)b->bufA;
            B.role[3] = (const T *)b->bufR0;
            B.red = b->dred;
            B.redn = b->dredn;
            B.r_phi = (T)tol.r_phi; B.a_phi = (T)tol.a_phi;
            B.r_c = (T)tol.r_c; B.a_c = (T)tol.a_c;
            e = launch_batch_euler<T>(b->N, B, b->nblocks, b->stream);
        }
        if (e == hipSuccess) e = launch_finalize_norm_batch(b->dred, b->dredn, b->dctl, n, b->dnorm, b->stream);
        b->norm_seq += 1.0;
        if (e == hipSuccess) e = launch_publish(b->dnorm, 3 * n, b->hnorm_dev, b->norm_seq, b->stream);
        if (e != hipSuccess) return bfail(b, PF_EHIP, "batch adaptive step: %s", hipGetErrorString(e));
        if ((rc = batch_wait_norms(b, b->norm_seq))) return rc;
        int accepted = 0;
        for (int i = 0; i < n; ++i) {
            if (!ctl[4 * i + 2]) continue;
            const double err = b->hnorm[3 * i + 2];
            bool acc;
            const double hn = ctrl_update(ctrl[i], 2, err, h[i], acc);
            st[i].rhs_evals += ns[i] + 1;
            st[i].stages += ns[i];
            st[i].last_err = err;
            if (acc) {
                ctl[4 * i + 3] = 1;
                ++accepted;
                b->t[i] = last[i] ? t_end[i] : b->t[i] + h[i];
                st[i].accepted++;
                st[i].last_dt = h[i];
                nonfinite[i] = 0;
            } else {
                st[i].rejected++;
                if (!std::isfinite(err) && ++nonfinite[i] >= 3 && !fail_rc)
                    fail_rc = bfail(b, PF_ENONFINITE, "instance %d: non-finite error norm three times in a row", i);
            }
            dt[i] = hn;
        }
        if (accepted) {
            BHIPCHK(b, hipMemcpyAsync(b->dctl, ctl.data(), sizeof(int) * 4 * n, hipMemcpyHostToDevice,
                                      b->stream));
            e = launch_batch_accept<T>((const T *)b->bufY, (T *)b->bufA, b->dlen, b->dlen + n, b->dctl, n,
                                       max_len, b->stream);
            if (e != hipSuccess) return bfail(b, PF_EHIP, "batch accept: %s", hipGetErrorString(e));
        }
        // the host tables are rewritten next step: their copies must be done
        BHIPCHK(b, hipStreamSynchronize(b->stream));
    }
    if (stats)
        for (int i = 0; i < n; ++i) {
            stats[i] = st[i];
            stats[i].t = b->t[i];
        }
    return fail_rc;
}

template <typename T>
pf_status batch_run(pf_batch *b, int integ, const double *t_end, const double *dt, int graph_k,
                    pf_stats *stats) {
    pf_status rc;
    if (integ == PF_RKL2 && (rc = batch_rkl2_buffers<T>(b))) return rc;
    b->integ = integ;
    int S = 0, stages = 1;
    rc = batch_plan<T>(b, t_end, dt, S, stages);
    if (rc) return rc;
    const int zero = 0;
    BHIPCHK(b, hipMemcpyAsync(b->dstep, &zero, sizeof(int), hipMemcpyHostToDevice, b->stream));
    const bool rkl2 = integ == PF_RKL2;
    const int d = rkl2 ? 1 : b->depth;
    const int launches = (S + d - 1) / d;
    int done = 0;
    if (graph_k > 0 && launches >= graph_k) {
        if ((rc = batch_graph<T>(b, graph_k, stages))) return rc;
        for (; done + graph_k <= launches; done += graph_k)
            BHIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
    }
    if (launches - done > 0 && (rc = batch_launch_steps<T>(b, launches - done, stages))) return rc;
    // forward Euler: an instance that took part in an odd number of launches
    // ends in buffer B, copied back; RKL2 steps end in the state buffer
    std::vector<BatchInst<T>> I(b->n);
    BHIPCHK(b, hipMemcpyAsync(I.data(), b->dinst, sizeof(BatchInst<T>) * b->n, hipMemcpyDeviceToHost,
                              b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->n; ++i) {
        const size_t bytes = (size_t)b->meta[i].F * b->meta[i].V * b->esz;
        if (!rkl2 && (((I[i].nsteps + d - 1) / d) & 1))
            BHIPCHK(b, hipMemcpyAsync((char *)b->bufA + b->off[i] * b->esz,
                                      (char *)b->bufB + b->off[i] * b->esz, bytes,
                                      hipMemcpyDeviceToDevice, b->stream));
        if (I[i].nsteps > 0) b->t[i] = t_end[i];
        if (stats) {
            const long long nf = I[i].nfull, nc = I[i].nsteps - I[i].nfull;
            stats[i] = pf_stats{};
            stats[i].accepted = I[i].nsteps;
            stats[i].rhs_evals = stats[i].stages =
                rkl2 ? nf * I[i].s_full + nc * I[i].s_last : I[i].nsteps;
            stats[i].t = b->t[i];
            stats[i].last_dt = I[i].nsteps ? (double)(I[i].nfull < I[i].nsteps ? I[i].dt_last : I[i].dt) : 0.0;
        }
    }
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    return PF_OK;
}

// Picks the persistent grid size and the stage-fusion depth: one launch of
// every supported depth (two steps of every instance planned, buffer A only
// read) timed for several grid sizes; the fastest time per step wins.
template <typename T>
pf_status batch_autotune(pf_batch *b, int *best_blocks, double *best_ms) {
    std::vector<double> t_end(b->n), dt(b->n);
    for (int i = 0; i < b->n; ++i) {
        dt[i] = 0.9 * stable_dt(&b->meta[i]);
        t_end[i] = b->t[i] + 2.0 * dt[i];
    }
    int S = 0, stages = 1;
    b->integ = PF_FEULER;
    pf_status rc = batch_plan<T>(b, t_end.data(), dt.data(), S, stages);
    if (rc) return rc;
    const int cands[5] = {512, 1024, 2048, 4096, 8192};
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    double best = 1e300;
    int bb = b->nblocks, bd = b->depth;
    const int zero = 0;
    for (int d = 1; d <= 2; ++d) {
        if (!batch_depth_ok(b, d)) continue;
        for (int c : cands) {
            const int nb = std::min(c, (b->total_tiles + 7) / 8 * 8);
            BHIPCHK(b, hipMemcpyAsync(b->dstep, &zero, sizeof(int), hipMemcpyHostToDevice, b->stream));
            hipError_t e = launch_batch_euler<T>(b->N, batch_args<T>(b, 0, d), nb, b->stream);
            BHIPCHK(b, hipEventRecord(e0, b->stream));
            for (int r = 0; r < 5 && e == hipSuccess; ++r)
                e = launch_batch_euler<T>(b->N, batch_args<T>(b, 0, d), nb, b->stream);
            if (e != hipSuccess) return bfail(b, PF_EHIP, "batch launch: %s", hipGetErrorString(e));
            BHIPCHK(b, hipEventRecord(e1, b->stream));
            BHIPCHK(b, hipEventSynchronize(e1));
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            const double per_step = ms / 5.0 / d;
            if (per_step < best) {
                best = per_step;
                bb = nb;
                bd = d;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->nblocks = bb;
    b->depth = bd;
    if (best_blocks) *best_blocks = bb;
    if (best_ms) *best_ms = best;
    return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_batch_destroy(pf_batch *b) {
    if (!b) return PF_EINVAL;
    if (b->stream) hipStreamSynchronize(b->stream);
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->graph) hipGraphDestroy(b->graph);
    void *ptrs[16] = {b->bufA, b->bufB, b->dparams, b->dinst, b->dtile, b->dstep,
                      b->bufQ2, b->bufS0, b->bufR0, b->dcoef, b->bufY, b->dred,
                      b->dredn, b->dnorm, b->dctl, b->dlen};
    for (void *q : ptrs)
        if (q) hipFree(q);
    if (b->hnorm) hipHostFree(b->hnorm);
    if (b->own_stream && b->stream) hipStreamDestroy(b->stream);
    delete b;
    return PF_OK;
}

pf_status pf_batch_create(const pf_params *per_inst, int n, pf_batch **out) {
    if (!per_inst || !out || n < 1) return PF_EINVAL;
    *out = nullptr;
    pf_batch *b = new (std::nothrow) pf_batch();
    if (!b) return PF_ENOMEM;
    b->n = n;
    b->meta.resize(n);
    pf_status rc = PF_OK;
    for (int i = 0; i < n && !rc; ++i) {
        rc = init_meta(&b->meta[i], &per_inst[i]);
        if (!rc && (per_inst[i].dim != 2 || per_inst[i].n_phi != per_inst[0].n_phi ||
                    per_inst[i].prec != per_inst[0].prec ||
                    (per_inst[i].with_c != 0) != (per_inst[0].with_c != 0)))
            rc = PF_EINVAL;  // instances share dim 2, N, precision and with_c
        // the batch kernel addresses an instance's whole state as one buffer group
        if (!rc && (unsigned long long)b->meta[i].F * b->meta[i].V * b->meta[i].esz > 0xFFFFFFFFull)
            rc = PF_EUNSUPPORTED;
        if (!rc && b->meta[i].walls) rc = PF_EUNSUPPORTED;  // batches are periodic
    }
    if (rc) {
        delete b;
        return rc;
    }
    b->N = b->meta[0].N;
    b->F = b->meta[0].F;
    b->with_c = b->meta[0].with_c;
    b->prec = b->meta[0].prec;
    b->esz = b->meta[0].esz;
    b->off.resize(n);
    b->ntx.resize(n);
    b->nty.resize(n);
    b->tile0.resize(n);
    b->t.assign(n, 0.0);
    b->have.assign(n, 0);
    std::vector<int> tile_inst;
    for (int i = 0; i < n; ++i) {
        b->off[i] = b->total;
        b->total += (long long)b->meta[i].F * b->meta[i].V;
        b->total = (b->total + 63) / 64 * 64;  // 256-byte aligned instance starts
        b->ntx[i] = (b->meta[i].nx + TILE_X - 1) / TILE_X;
        b->nty[i] = (b->meta[i].ny + tile_rows(2, b->meta[i].N) - 1) / tile_rows(2, b->meta[i].N);
        b->tile0[i] = b->total_tiles;
        b->total_tiles += b->ntx[i] * b->nty[i];
        tile_inst.insert(tile_inst.end(), (size_t)b->ntx[i] * b->nty[i], i);
    }
    if (hipMalloc(&b->bufA, b->total * b->esz) != hipSuccess ||
        hipMalloc(&b->bufB, b->total * b->esz) != hipSuccess ||
        hipMalloc(&b->dtile, sizeof(int) * tile_inst.size()) != hipSuccess ||
        hipMalloc(&b->dstep, sizeof(int)) != hipSuccess) {
        pf_batch_destroy(b);
        return PF_ENOMEM;
    }
    if (hipMemcpy(b->dtile, tile_inst.data(), sizeof(int) * tile_inst.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(b->bufA, 0, b->total * b->esz) != hipSuccess) {
        pf_batch_destroy(b);
        return PF_EHIP;
    }
    rc = b->prec == PF_FP64 ? batch_setup_params<double>(b) : batch_setup_params<float>(b);
    if (!rc && hipStreamCreate(&b->stream) != hipSuccess) rc = PF_EHIP;
    if (rc) {
        pf_batch_destroy(b);
        return rc;
    }
    b->own_stream = true;
    b->nblocks = std::min(2048, (b->total_tiles + 7) / 8 * 8);
    *out = b;
    return PF_OK;
}

pf_status pf_batch_set_stream(pf_batch *b, void *stream) {
    if (!b || !stream) return PF_EINVAL;  // graph capture needs a real stream
    // the batch's work queued on the previous stream ends before any of its
    // work on the next one starts
    if ((hipStream_t)stream != b->stream && hipStreamSynchronize(b->stream) != hipSuccess)
        return bfail(b, PF_EHIP, "hipStreamSynchronize of the previous stream failed");
    if (b->own_stream) {
        hipStreamDestroy(b->stream);
        b->own_stream = false;
    }
    b->stream = (hipStream_t)stream;
    return PF_OK;
}

pf_status pf_batch_init_fields(pf_batch *b, int i, const double *u, double t0) {
    if (!b || !u || i < 0 || i >= b->n) return PF_EINVAL;
    const long long n = (long long)b->meta[i].F * b->meta[i].V;
    if (b->prec == PF_FP64) {
        BHIPCHK(b, hipMemcpyAsync((double *)b->bufA + b->off[i], u, n * sizeof(double),
                                  hipMemcpyHostToDevice, b->stream));
    } else {
        std::vector<float> h(n);
        for (long long k = 0; k < n; ++k) h[k] = (float)u[k];
        BHIPCHK(b, hipMemcpyAsync((float *)b->bufA + b->off[i], h.data(), n * sizeof(float),
                                  hipMemcpyHostToDevice, b->stream));
    }
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->t[i] = t0;
    b->have[i] = 1;
    return PF_OK;
}

pf_status pf_batch_get_fields(pf_batch *b, int i, double *u, double *t) {
    if (!b || i < 0 || i >= b->n) return PF_EINVAL;
    if (!b->have[i]) return bfail(b, PF_ESTATE, "instance %d has no fields", i);
    if (t) *t = b->t[i];
    if (!u) return PF_OK;
    const long long n = (long long)b->meta[i].F * b->meta[i].V;
    if (b->prec == PF_FP64) {
        BHIPCHK(b, hipMemcpyAsync(u, (double *)b->bufA + b->off[i], n * sizeof(double),
                                  hipMemcpyDeviceToHost, b->stream));
        BHIPCHK(b, hipStreamSynchronize(b->stream));
    } else {
        std::vector<float> h(n);
        BHIPCHK(b, hipMemcpyAsync(h.data(), (float *)b->bufA + b->off[i], n * sizeof(float),
                                  hipMemcpyDeviceToHost, b->stream));
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        for (long long k = 0; k < n; ++k) u[k] = (double)h[k];
    }
    return PF_OK;
}

pf_status pf_batch_stable_dt(pf_batch *b, int i, double *dte) {
    if (!b || !dte || i < 0 || i >= b->n) return PF_EINVAL;
    *dte = stable_dt(&b->meta[i]);
    return PF_OK;
}

pf_status pf_batch_run_to(pf_batch *b, pf_integrator integ, const double *t_end, const double *dt,
                          int graph_steps, pf_stats *stats) {
    if (!b || !t_end || graph_steps < 0) return PF_EINVAL;
    if (integ != PF_FEULER && integ != PF_RKL2)
        return bfail(b, PF_EUNSUPPORTED, "the batch advances forward Euler or RKL2 steps");
    for (int i = 0; i < b->n; ++i) {
        if (!b->have[i]) return bfail(b, PF_ESTATE, "instance %d has no fields", i);
        if (!std::isfinite(t_end[i])) return bfail(b, PF_EINVAL, "instance %d: t_end must be finite", i);
    }
    return b->prec == PF_FP64 ? batch_run<double>(b, integ, t_end, dt, graph_steps, stats)
                              : batch_run<float>(b, integ, t_end, dt, graph_steps, stats);
}

pf_status pf_batch_run_adaptive(pf_batch *b, pf_integrator integ, const double *t_end,
                                const pf_tol *tol, pf_stats *stats) {
    if (!b || !t_end || !tol) return PF_EINVAL;
    if (integ != PF_RKL2) return bfail(b, PF_EUNSUPPORTED, "adaptive batches take RKL2 steps");
    if (b->n > 65535) return bfail(b, PF_EUNSUPPORTED, "adaptive batches hold at most 65535 instances");
    if (!(tol->r_phi >= 0.0 && tol->a_phi >= 0.0 && tol->r_c >= 0.0 && tol->a_c >= 0.0) ||
        !(tol->a_phi > 0.0 || tol->r_phi > 0.0) || !(tol->a_c > 0.0 || tol->r_c > 0.0))
        return bfail(b, PF_EINVAL, "tolerances must be >= 0 with a nonzero weight per field kind");
    for (int i = 0; i < b->n; ++i) {
        if (!b->have[i]) return bfail(b, PF_ESTATE, "instance %d has no fields", i);
        if (!(t_end[i] >= b->t[i]) || !std::isfinite(t_end[i]))
            return bfail(b, PF_EINVAL, "instance %d: t_end before t or not finite", i);
    }
    return b->prec == PF_FP64 ? batch_run_adaptive<double>(b, t_end, *tol, stats)
                              : batch_run_adaptive<float>(b, t_end, *tol, stats);
}

pf_status pf_batch_autotune(pf_batch *b, int *nblocks, double *best_ms) {
    if (!b) return PF_EINVAL;
    for (int i = 0; i < b->n; ++i)
        if (!b->have[i]) return bfail(b, PF_ESTATE, "instance %d has no fields", i);
    return b->prec == PF_FP64 ? batch_autotune<double>(b, nblocks, best_ms)
                              : batch_autotune<float>(b, nblocks, best_ms);
}

pf_status pf_batch_set_blocks(pf_batch *b, int nblocks) {
    if (!b || nblocks < 8) return PF_EINVAL;
    b->nblocks = nblocks / 8 * 8;
    return PF_OK;
}

pf_status pf_batch_set_fusion(pf_batch *b, int depth) {
    if (!b || (depth != 1 && depth != 2)) return PF_EINVAL;
    if (!batch_depth_ok(b, depth))
        return bfail(b, PF_EUNSUPPORTED, "fusion depth %d needs more LDS than a workgroup has at N = %d",
                     depth, b->N);
    b->depth = depth;
    return PF_OK;
}

pf_status pf_batch_get_config(const pf_batch *b, int *nblocks, int *depth) {
    if (!b) return PF_EINVAL;
    if (nblocks) *nblocks = b->nblocks;
    if (depth) *depth = b->depth;
    return PF_OK;
}

const char *pf_batch_last_error(const pf_batch *b) { return b ? b->err.c_str() : "null handle"; }

}  // extern "C"
