// pf_host_check -- host-memory check of libpf's C-ABI.  The build links this
// program with the host engine compiled under AddressSanitizer (host code
// only; the device code is the ordinary build) and it calls every entry point
// with exactly sized heap arrays, ragged sizes and invalid arguments, so that
// a read or write past an array, a use after free or a leak in the engine's
// host code stops the run.
//
//   pf_host_check host   calls that need no GPU (argument checks, the host
//                        helpers, the host error norm); pf_create of a valid
//                        parameter set must fail cleanly without a device
//   pf_host_check gpu    additionally runs handles and a batch on device 0
//
// Prints one line per section and "ok" at the end; every failed check is
// printed and makes the exit status 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pf.h"

static int fails = 0;
#define EXPECT(cond, ...)                                         \
    do {                                                          \
        if (!(cond)) {                                            \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                    \
            std::fprintf(stderr, "\n");                           \
            ++fails;                                              \
        }                                                         \
    } while (0)

// exactly sized heap arrays: one element past the end is a red zone
template <typename T>
static T *exact(size_t n) {
    return static_cast<T *>(std::malloc(n ? n * sizeof(T) : 1));
}

static unsigned long long rng = 0x9e3779b97f4a7c15ull;
static double urand() {  // splitmix64, uniform in [0, 1)
    unsigned long long z = (rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct Model {
    std::vector<int> type_of;
    std::vector<double> gamma, mob, k, c0, D;
    pf_params p;
    Model(int dim, int n, int nphi, int with_c, pf_precision prec) {
        const int nt = 2;
        type_of.resize(nphi);
        for (int a = 0; a < nphi; ++a) type_of[a] = a == nphi - 1 && nphi > 2 ? 1 : 0;
        gamma = {1.0, 1.0, 1.0, 1.2};
        mob = {1.0, 0.5, 0.5, 0.25};
        k = {1.0, 2.0};
        c0 = {0.1, 0.9};
        D = {1.0, 0.1};
        std::memset(&p, 0, sizeof p);
        p.dim = dim;
        p.nx = n;
        p.ny = n - 3;  // ragged: not a multiple of the tile
        p.nz = dim == 3 ? n - 5 : 1;
        p.dx = 1.0;
        p.W = 2.5;
        p.n_phi = nphi;
        p.type_of = type_of.data();
        p.n_types = nt;
        p.gamma = gamma.data();
        p.mob = mob.data();
        p.k = k.data();
        p.c0 = c0.data();
        p.D = D.data();
        p.with_c = with_c;
        p.prec = prec;
        p.ssp_stages = 3;
    }
    long long V() const { return (long long)p.nx * p.ny * p.nz; }
    int F() const { return p.n_phi + (p.with_c != 0); }
};

// phases on the simplex: a few disks of different phases over phase 0
static void fill_state(const pf_params &p, double *u) {
    const long long V = (long long)p.nx * p.ny * p.nz;
    const int N = p.n_phi;
    std::memset(u, 0, sizeof(double) * (size_t)(N + (p.with_c != 0)) * V);
    for (long long i = 0; i < V; ++i) u[i] = 1.0;
    for (int a = 1; a < N; ++a) {
        const double cx = urand() * p.nx, cy = urand() * p.ny, cz = urand() * p.nz;
        const double r = 2.0 + 3.0 * urand();
        for (int z = 0; z < p.nz; ++z)
            for (int y = 0; y < p.ny; ++y)
                for (int x = 0; x < p.nx; ++x) {
                    const double d = std::sqrt((x - cx) * (x - cx) + (y - cy) * (y - cy) +
                                               (p.dim == 3 ? (z - cz) * (z - cz) : 0.0));
                    double v = 0.5 - (d - r) / (M_PI * p.W);
                    v = v < 0 ? 0 : (v > 1 ? 1 : v);
                    const long long i = ((long long)z * p.ny + y) * p.nx + x;
                    const double take = v * u[i];
                    u[i] -= take;
                    u[(long long)a * V + i] += take;
                }
    }
    if (p.with_c)
        for (long long i = 0; i < V; ++i) u[(long long)N * V + i] = 0.1 + 0.8 * u[(long long)(N - 1) * V + i];
}

static void host_section() {
    // supported N
    int cnt = pf_supported_nphi(nullptr, 0);
    EXPECT(cnt > 0, "pf_supported_nphi count %d", cnt);
    for (int cap = 0; cap <= cnt + 1; ++cap) {
        int *buf = exact<int>(cap);
        EXPECT(pf_supported_nphi(cap ? buf : nullptr, cap) == cnt, "cap %d", cap);
        std::free(buf);
    }
    std::printf("supported_nphi: %d values\n", cnt);

    // parameter validation on pf_params_stable_dt and pf_create
    Model m(2, 24, 3, 1, PF_FP64);
    double dte = 0;
    EXPECT(pf_params_stable_dt(&m.p, &dte) == PF_OK && dte > 0, "valid stable dt");
    EXPECT(pf_params_stable_dt(nullptr, &dte) == PF_EINVAL, "null params");
    EXPECT(pf_params_stable_dt(&m.p, nullptr) == PF_EINVAL, "null out");
    int bad = 0;
    for (int v = 0; v < 20; ++v) {
        Model b(2, 24, 3, 1, PF_FP64);
        std::vector<int> tbad(b.type_of);
        switch (v) {
        case 0: b.p.n_phi = 0; break;
        case 1: b.p.n_phi = 1; break;
        case 2: b.p.n_phi = 17; break;
        case 3: tbad[1] = 2; b.p.type_of = tbad.data(); break;
        case 4: tbad[0] = -1; b.p.type_of = tbad.data(); break;
        case 5: b.p.n_types = 0; break;
        case 6: b.p.n_types = 5; break;
        case 7: b.p.nx = 0; break;
        case 8: b.p.dim = 4; break;
        case 9: b.p.nz = 2; break;
        case 10: b.p.dx = -1.0; break;
        case 11: b.gamma[1] = NAN; break;
        case 12: b.p.bc[0] = 2; break;
        case 13: b.p.c_fixed[0] = 1; break;  // fixed c on a periodic axis
        case 14: b.p.ssp_stages = 1; break;
        case 15: b.p.W = 0.0; break;
        case 16: b.p.type_of = nullptr; break;
        case 17: b.p.bc[2] = 1; break;  // walls on z of a 2D grid
        case 18: b.p.bc[0] = 1; b.p.c_fixed[1] = 1; b.p.c_bc[1] = INFINITY; break;
        case 19: b.p.nx = b.p.ny = 1 << 20; break;  // too large to address
        }
        pf_sim *s = reinterpret_cast<pf_sim *>(&m);  // must be overwritten with NULL
        const pf_status rc = pf_create(&b.p, &s);
        EXPECT(rc < 0 && s == nullptr, "invalid parameter set %d: rc %d", v, rc);
        EXPECT(pf_params_stable_dt(&b.p, &dte) < 0, "stable dt of set %d", v);
        bad += rc < 0;
    }
    std::printf("parameter checks: %d invalid sets refused\n", bad);

    // RKL stage counts over a wide range of dt / dt_e
    int s = 0, last = 0;
    for (double r = 1e-3; r < 1e5; r *= 1.37) {
        EXPECT(pf_rkl_stage_count(PF_RKL2, r, 1.0, &s) == PF_OK && s >= 1 && (s & 1), "rkl2 %g", r);
        EXPECT(s >= last, "non-monotone stage count");
        last = s;
        EXPECT(pf_rkl_stage_count(PF_RKL1, r, 1.0, &s) == PF_OK && s >= 1, "rkl1 %g", r);
    }
    EXPECT(pf_rkl_stage_count(PF_FEULER, 1.0, 1.0, &s) == PF_EINVAL, "fe stage count");
    EXPECT(pf_rkl_stage_count(PF_RKL2, 0.0, 1.0, &s) == PF_EINVAL, "dt 0");
    EXPECT(pf_rkl_stage_count(PF_RKL2, NAN, 1.0, &s) == PF_EINVAL, "dt nan");
    EXPECT(pf_rkl_stage_count(PF_RKL2, 1.0, -1.0, &s) == PF_EINVAL, "dte < 0");
    EXPECT(pf_rkl_stage_count(PF_RKL2, 1.0, 1.0, nullptr) == PF_EINVAL, "null s");
    std::printf("stage counts: up to %d stages\n", last);

    // controller over random, tiny, huge and non-finite errors
    pf_controller c;
    EXPECT(pf_controller_init(&c) == PF_OK, "controller init");
    EXPECT(pf_controller_init(nullptr) == PF_EINVAL, "controller init null");
    double h = 1.0;
    int acc = 0, nacc = 0;
    const double specials[] = {0.0, 1e-300, 1e300, INFINITY, NAN, 1.0, 0.999999};
    for (int i = 0; i < 20000; ++i) {
        double e = i % 11 == 0 ? specials[(i / 11) % 7] : std::exp(8.0 * (urand() - 0.5));
        double hn = 0;
        const int order = 1 + i % 4;
        EXPECT(pf_controller_update(&c, order, e, h, &acc, &hn) == PF_OK, "update %d", i);
        EXPECT(std::isfinite(hn) && hn > 0 && (acc == 0 || acc == 1), "h_next %g at e %g", hn, e);
        nacc += acc;
        h = hn < 1e-200 || hn > 1e200 ? 1.0 : hn;
    }
    double hn = 0;
    EXPECT(pf_controller_update(nullptr, 2, 0.5, 1.0, &acc, &hn) == PF_EINVAL, "update null");
    std::printf("controller: %d of 20000 accepted\n", nacc);

    // exact output times
    double hu = 0;
    EXPECT(pf_clip_step(0.0, 1.0, 0.3, &hu, &last) == 1 && hu == 0.3 && !last, "clip");
    EXPECT(pf_clip_step(0.9, 1.0, 0.3, &hu, &last) == 1 && last, "clip last");
    EXPECT(pf_clip_step(1.0, 1.0, 0.3, &hu, &last) == 0, "clip end");
    EXPECT(pf_clip_step(0.0, 1.0, 0.0, &hu, &last) == -1, "clip h 0");
    EXPECT(pf_clip_step(0.0, 1.0, NAN, &hu, &last) == -1, "clip nan");
    EXPECT(pf_clip_step(0.0, 1.0, 0.3, nullptr, &last) == -1, "clip null");

    // host error norm over every N, with and without c, ragged cell counts
    int norms = 0;
    for (int nphi = 1; nphi <= 16; ++nphi)
        for (int wc = 0; wc <= 1; ++wc)
            for (long long cells : {1LL, 2LL, 3LL, 7LL, 64LL, 65LL, 257LL}) {
                Model mm(2, 8, nphi < 2 ? 2 : nphi, wc, PF_FP64);
                mm.p.n_phi = nphi;  // only n_phi and with_c are read
                const size_t n = (size_t)(nphi + wc) * cells;
                double *e = exact<double>(n), *u0 = exact<double>(n), *u1 = exact<double>(n);
                for (size_t i = 0; i < n; ++i) {
                    e[i] = urand() < 0.3 ? 0.0 : 1e-3 * (urand() - 0.5);
                    u0[i] = urand();
                    u1[i] = urand();
                }
                pf_tol tol = {1e-4, 1e-2, 1e-4, 1e-4, 200.0, 0.0};
                double out = -1;
                EXPECT(pf_error_norm(&mm.p, cells, e, u0, u1, &tol, &out) == PF_OK && std::isfinite(out) &&
                           out >= 0,
                       "norm n_phi %d c %d cells %lld", nphi, wc, cells);
                norms++;
                std::free(e);
                std::free(u0);
                std::free(u1);
            }
    {
        double x = 0, out = 0;
        pf_tol tol = {1e-4, 1e-2, 1e-4, 1e-4, 200.0, 0.0};
        pf_tol neg = {-1e-4, 1e-2, 1e-4, 1e-4, 200.0, 0.0};
        EXPECT(pf_error_norm(&m.p, 0, &x, &x, &x, &tol, &out) == PF_EINVAL, "norm cells 0");
        EXPECT(pf_error_norm(&m.p, 1, nullptr, &x, &x, &tol, &out) == PF_EINVAL, "norm null e");
        EXPECT(pf_error_norm(&m.p, 1, &x, &x, &x, &neg, &out) == PF_EINVAL, "norm negative tol");
        EXPECT(pf_error_norm(nullptr, 1, &x, &x, &x, &tol, &out) == PF_EINVAL, "norm null params");
    }
    std::printf("host error norms: %d shapes\n", norms);

    // null handles
    EXPECT(pf_destroy(nullptr) == PF_EINVAL, "destroy null");
    EXPECT(pf_batch_destroy(nullptr) == PF_EINVAL, "batch destroy null");
    EXPECT(pf_last_error(nullptr) != nullptr, "last error null");
    EXPECT(pf_batch_last_error(nullptr) != nullptr, "batch last error null");
    pf_batch *b = nullptr;
    EXPECT(pf_batch_create(nullptr, 2, &b) == PF_EINVAL && !b, "batch null params");
    EXPECT(pf_batch_create(&m.p, 0, &b) == PF_EINVAL && !b, "batch n 0");
    EXPECT(pf_batch_create(&m.p, -3, &b) == PF_EINVAL && !b, "batch n < 0");
    int on = -1;
    EXPECT(pf_set_r0_recompute(nullptr, 1) == PF_EINVAL, "r0 recompute null");
    EXPECT(pf_get_r0_recompute(nullptr, &on) == PF_EINVAL && on == -1, "r0 recompute get null");
    std::printf("null handles: ok\n");
}

static void check_handle(int dim, int n, int nphi, int with_c, pf_precision prec) {
    Model m(dim, n, nphi, with_c, prec);
    const long long V = m.V();
    const int F = m.F();
    pf_sim *s = nullptr;
    pf_status rc = pf_create(&m.p, &s);
    EXPECT(rc == PF_OK && s, "create dim %d N %d: %d", dim, nphi, rc);
    if (!s) return;
    double *phi = exact<double>((size_t)nphi * V), *c = with_c ? exact<double>(V) : nullptr;
    double *u = exact<double>((size_t)F * V);
    fill_state(m.p, u);
    std::memcpy(phi, u, sizeof(double) * (size_t)nphi * V);
    if (with_c) std::memcpy(c, u + (size_t)nphi * V, sizeof(double) * V);
    EXPECT(pf_step(s, PF_FEULER, 0.1, nullptr) == PF_ESTATE, "step before init");
    EXPECT(pf_init_fields(s, phi, c, 0.0) == PF_OK, "init split");
    EXPECT(pf_init_fields(s, u, nullptr, 0.0) == PF_OK, "init joined");
    double dte = 0;
    EXPECT(pf_stable_dt(s, &dte) == PF_OK && dte > 0, "stable dt");
    pf_stats st;
    const pf_integrator ints[] = {PF_FEULER, PF_SSP_S2, PF_SSP_10_4, PF_RKL1, PF_RKL2};
    const double mult[] = {0.9, 1.5, 4.0, 12.0, 40.0};
    for (int i = 0; i < 5; ++i) EXPECT(pf_step(s, ints[i], mult[i] * dte, &st) == PF_OK, "step %d", i);
    pf_tol tol = {1e-4, 1e-2, 1e-4, 1e-4, 200.0, 0.0};
    double t = 0;
    EXPECT(pf_get_fields(s, phi, c, &t) == PF_OK, "get split");
    EXPECT(pf_run_to(s, PF_RKL2, t + 60 * dte, &tol, 0.0, &st) == PF_OK, "adaptive rkl2");
    EXPECT(pf_run_to(s, PF_SSP_10_4, st.t + 10 * dte, &tol, 0.0, &st) == PF_OK, "adaptive ssp104");
    EXPECT(pf_run_to(s, PF_RKL1, st.t + 30 * dte, nullptr, 7 * dte, &st) == PF_OK, "fixed rkl1");
    long long nt = 0;
    EXPECT(pf_get_trace(s, nullptr, 0, &nt) == PF_OK && nt > 0, "trace count");
    for (long long cap : {1LL, nt - 1, nt, nt + 3}) {
        double *tb = exact<double>((size_t)(4 * cap));
        long long n2 = 0;
        EXPECT(pf_get_trace(s, tb, cap, &n2) == PF_OK && n2 == nt, "trace cap %lld", cap);
        std::free(tb);
    }
    double *r = exact<double>((size_t)F * V);
    EXPECT(pf_rhs(s, r, with_c ? r + (size_t)nphi * V : nullptr) == PF_OK, "rhs");
    std::free(r);
    double d[5];
    EXPECT(pf_diagnostics(s, d) == PF_OK && d[4] == 0, "diagnostics");
    size_t len = 0;
    EXPECT(pf_get_state(s, nullptr, &len) == PF_OK && len > 0, "state size");
    unsigned char *ck = exact<unsigned char>(len);
    EXPECT(pf_get_state(s, ck, &len) == PF_OK, "get state");
    EXPECT(pf_set_state(s, ck, len - 1) == PF_EINVAL, "short state");
    EXPECT(pf_set_state(s, ck, len) == PF_OK, "set state");
    std::free(ck);
    int tx = 0, zc = 0;
    double best = 0;
    EXPECT(pf_autotune(s, &tx, &zc, &best) == PF_OK && best > 0, "autotune");
    EXPECT(pf_set_tiling(s, 64, 3) == PF_OK, "tiling");
    EXPECT(pf_step(s, PF_RKL2, 30 * dte, nullptr) == PF_OK, "step after tiling");
    EXPECT(pf_get_fields(s, u, nullptr, &t) == PF_OK, "get joined");
    EXPECT(pf_set_timing(s, 1) == PF_OK, "timing on");
    EXPECT(pf_step(s, PF_RKL2, 30 * dte, nullptr) == PF_OK, "timed step");
    double ms = 0;
    long long launches = 0;
    EXPECT(pf_get_kernel_time(s, 0, &ms, &launches) == PF_OK && launches > 0, "kernel time");
    EXPECT(pf_set_timing(s, 0) == PF_OK, "timing off");
    {
        // R0 recomputed in the 3D inner stages: same bits as the stored R0
        const bool built = dim == 3 && (prec == PF_FP32 ? nphi <= 9 : nphi <= 4);
        int on = -1;
        EXPECT(pf_set_r0_recompute(s, 2) == PF_EINVAL, "r0 recompute 2");
        EXPECT(pf_get_r0_recompute(s, nullptr) == PF_EINVAL, "r0 recompute get null out");
        EXPECT(pf_set_r0_recompute(s, 1) == (built ? PF_OK : PF_EUNSUPPORTED), "r0 recompute on");
        EXPECT(pf_get_r0_recompute(s, &on) == PF_OK && on == (built ? 1 : 0), "r0 recompute get");
        if (built) {
            fill_state(m.p, u);
            EXPECT(pf_init_fields(s, u, nullptr, 0.0) == PF_OK, "rc init");
            EXPECT(pf_step(s, PF_RKL2, 30 * dte, nullptr) == PF_OK, "rc step");
            double *u1 = exact<double>((size_t)F * V), *u2 = exact<double>((size_t)F * V);
            EXPECT(pf_get_fields(s, u1, nullptr, &t) == PF_OK, "rc get");
            EXPECT(pf_set_r0_recompute(s, 0) == PF_OK, "r0 recompute off");
            EXPECT(pf_init_fields(s, u, nullptr, 0.0) == PF_OK, "stored init");
            EXPECT(pf_step(s, PF_RKL2, 30 * dte, nullptr) == PF_OK, "stored step");
            EXPECT(pf_get_fields(s, u2, nullptr, &t) == PF_OK, "stored get");
            EXPECT(std::memcmp(u1, u2, sizeof(double) * (size_t)F * V) == 0, "rc equals stored R0");
            std::free(u1);
            std::free(u2);
        }
    }
    if (nphi <= 8) {
        EXPECT(pf_set_sparse_storage(s, nphi < 4 ? nphi : 4) == PF_OK, "sparse on");
        fill_state(m.p, u);
        EXPECT(pf_init_fields(s, u, nullptr, 0.0) == PF_OK, "sparse init");
        EXPECT(pf_step(s, PF_RKL2, 20 * dte, nullptr) == PF_OK, "sparse step");
        EXPECT(pf_get_fields(s, u, nullptr, &t) == PF_OK, "sparse get");
        long long cuts = -1;
        EXPECT(pf_sparse_cuts(s, &cuts) == PF_OK && cuts >= 0, "sparse cuts");
        EXPECT(pf_set_sparse_storage(s, 0) == PF_OK, "sparse off");
    }
    EXPECT(pf_destroy(s) == PF_OK, "destroy");
    std::free(phi);
    std::free(c);
    std::free(u);
    std::printf("handle dim %d N %d c %d %s: ok\n", dim, nphi, with_c, prec == PF_FP64 ? "fp64" : "fp32");
}

static void check_batch() {
    const int n = 3;
    std::vector<Model> ms;
    for (int i = 0; i < n; ++i) ms.emplace_back(2, 20 + 7 * i, 3, 1, PF_FP32);
    std::vector<pf_params> ps;
    for (auto &mm : ms) ps.push_back(mm.p);
    pf_batch *b = nullptr;
    EXPECT(pf_batch_create(ps.data(), n, &b) == PF_OK && b, "batch create");
    if (!b) return;
    std::vector<double *> us;
    for (int i = 0; i < n; ++i) {
        double *u = exact<double>((size_t)ms[i].F() * ms[i].V());
        fill_state(ms[i].p, u);
        EXPECT(pf_batch_init_fields(b, i, u, 0.0) == PF_OK, "batch init %d", i);
        us.push_back(u);
    }
    EXPECT(pf_batch_init_fields(b, n, us[0], 0.0) == PF_EINVAL, "batch index out of range");
    double *te = exact<double>(n), *dts = exact<double>(n);
    pf_stats *st = exact<pf_stats>(n);
    for (int i = 0; i < n; ++i) {
        double dte = 0;
        EXPECT(pf_batch_stable_dt(b, i, &dte) == PF_OK, "batch dte");
        dts[i] = 0.9 * dte;
        te[i] = 25.5 * dts[i];
    }
    EXPECT(pf_batch_run_to(b, PF_FEULER, te, dts, 0, st) == PF_OK, "batch fe");
    for (int i = 0; i < n; ++i) te[i] += 40 * dts[i];
    EXPECT(pf_batch_run_to(b, PF_FEULER, te, nullptr, 4, st) == PF_OK, "batch fe graph");
    for (int i = 0; i < n; ++i) {
        dts[i] *= 30;
        te[i] += 3.5 * dts[i];
    }
    EXPECT(pf_batch_run_to(b, PF_RKL2, te, dts, 0, st) == PF_OK, "batch rkl2");
    for (int i = 0; i < n; ++i) te[i] += 3 * dts[i];
    EXPECT(pf_batch_run_to(b, PF_RKL2, te, dts, 2, st) == PF_OK, "batch rkl2 graph");
    pf_tol tol = {1e-4, 1e-2, 1e-4, 1e-4, 200.0, 0.0};
    for (int i = 0; i < n; ++i) te[i] += 2 * dts[i];
    EXPECT(pf_batch_run_adaptive(b, PF_RKL2, te, &tol, st) == PF_OK, "batch adaptive");
    int nb = 0, depth = 0;
    double best = 0;
    EXPECT(pf_batch_autotune(b, &nb, &best) == PF_OK && nb > 0, "batch autotune");
    EXPECT(pf_batch_get_config(b, &nb, &depth) == PF_OK, "batch config");
    for (int i = 0; i < n; ++i) {
        double t = 0;
        EXPECT(pf_batch_get_fields(b, i, us[i], &t) == PF_OK && t == te[i], "batch get %d", i);
        std::free(us[i]);
    }
    EXPECT(pf_batch_destroy(b) == PF_OK, "batch destroy");
    std::free(te);
    std::free(dts);
    std::free(st);
    std::printf("batch of %d: ok\n", n);
}

int main(int argc, char **argv) {
    const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
    host_section();
    Model m(2, 24, 3, 1, PF_FP64);
    pf_sim *s = nullptr;
    const pf_status rc = pf_create(&m.p, &s);
    if (!gpu) {
        // without a device the valid handle cannot be made: a clean failure
        EXPECT(rc < 0 && s == nullptr, "create without a device: %d", rc);
        if (s) pf_destroy(s);
    } else {
        EXPECT(rc == PF_OK && s, "create: %d", rc);
        if (s) pf_destroy(s);
        check_handle(2, 40, 3, 1, PF_FP64);
        check_handle(2, 70, 4, 1, PF_FP32);
        check_handle(2, 36, 8, 0, PF_FP32);
        check_handle(3, 20, 3, 1, PF_FP64);
        check_handle(3, 24, 9, 1, PF_FP32);
        check_batch();
    }
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
