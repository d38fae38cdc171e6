// pf_internal.h -- structures shared by the gfx950 kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pf {

constexpr int NMAX = 16;  // largest number of order parameters a kernel is built for
constexpr int TMAX = 4;   // largest number of thermodynamic types
// Stage kernel blocks are 256 threads.  2D: 64 threads per row (one
// wavefront per row of 64 cells), TILE_Y = 4 rows of threads.
constexpr int TILE_X = 64, TILE_Y = 4;
// Cells per thread in y of a 2D tile with n order parameters: the tile is
// 64 x (4 rows2d(n)) cells, each thread computing rows2d(n) cells of one
// column.  Two rows halve the barriers and the halo share per cell (the halo
// is loaded and its mu and Mc computed by the same 256 threads); for few
// fields that is instruction time saved, while for eight or more fields the
// second row's values cost the kernels a wave per SIMD, so they keep one row.
constexpr int ROWS2D_MAX_N = 4;
constexpr int rows2d(int n) { return n <= ROWS2D_MAX_N ? 2 : 1; }
// A 3D tile is TILE3_X x TILE3_Y cells, one per thread, marched in z.  The
// build may choose 32 x 8 (-DPF_TILE3_X=32: half the y-halo per cell, rows of
// 32 cells still whole 128-byte lines) instead of 64 x 4; on the 512^3 N = 9
// workload both run at the streaming rate of their own access pattern and
// 64 x 4 measured marginally faster, so it is the default.
#ifndef PF_TILE3_X
#define PF_TILE3_X 64
#endif
constexpr int TILE3_X = PF_TILE3_X, TILE3_Y = 256 / PF_TILE3_X;
constexpr int tile_cols(int dim) { return dim == 3 ? TILE3_X : TILE_X; }
constexpr int thread_rows(int dim) { return 256 / tile_cols(dim); }
constexpr int tile_rows(int dim, int n) { return dim == 2 ? TILE_Y * rows2d(n) : TILE3_Y; }
// Largest number of order parameters built with stage-fusion depth 2.
constexpr int DEPTH2_MAX_N = 4;

// Per-simulation constants, resident in device memory and read through the
// scalar cache (every address is uniform across the wavefront).  Pair tables
// are full n_phi x n_phi, row-major; per-phase tables are indexed by phase.
template <typename T>
struct DevParams {
    int nx, ny, nz, n_phi, with_c, n_types;
    long long V;   // cells per plane-field (nx*ny*nz)
    T idx2;        // 1/dx^2
    T A[NMAX * NMAX];
    T B[NMAX * NMAX];
    T L[NMAX * NMAX];
    T c0[NMAX];    // c0 of the phase's type
    T ik[NMAX];    // 1/k of the phase's type
    T Dk[NMAX];    // D/k of the phase's type
    T k2[NMAX];    // 2k of the phase's type
    T hik[NMAX];   // 1/(2k) of the phase's type
    int tphi[NMAX];
    int uniform;   // 1 when every pair (a != b) has the same A, B and L
    int walls;     // bit a: axis a (x, y, z) ends in zero-gradient walls
    int cfix;      // bit f: face f (x-, x+, y-, y+, z-, z+) holds c at cbc[f]
    T cbc[6];
    T k2t[TMAX];   // 2k per type (grand potential)
    T hikt[TMAX];  // 1/(2k) per type
    T c0t[TMAX];   // c0 per type
    T ikt[TMAX];   // 1/k per type
    T Dkt[TMAX];   // D/k per type
};

// Stage kinds of the fused stencil kernel.  Each evaluates rhs(y1) at the
// cell (eqs. phieq, ceq), forms one stage combination and projects the phi
// planes onto the simplex (except RHS and EST, which project nothing).
enum StageKind : int {
    K_RHS = 0,          // out = rhs(y1)
    K_EULER = 1,        // out = S(y1 + a r), or S(y1 + a (r / b)) when b != 0 (the
                        // SSP(s)2 sub-step of Alg. ssp2); out2 (optional) = r
    K_SSP2_FINAL = 2,   // out = S(((a y1 + u0) + b r) / c)
    K_SSP104_S5 = 3,    // y = S(y1 + a r); out2 = b u0 + c y; out = S(d out2 - e y);
                        // FP32: out2 = y, out = S(u0 + f (y - u0))
    K_SSP104_FINAL = 4, // out = S((u0 + a y1) + b r);
                        // FP32: S(y2 + c (u0 - y2) + a (y1 - y2) + b r), y2 = u^n
    K_RKL1 = 5,         // out = S((a y1 + b y2) + c r); FP32: S(y1 + b (y2 - y1) + c r), a + b = 1
    K_RKL2_FIRST = 6,   // y* = y1 + a r; out = S(y*); out2 = R0 (corrected where S acted)
    K_RKL2 = 7,         // out = S(((a u0 + b y1) + c y2) + d ((e r) + (f r0)));
                        // FP32: u0 + b (y1 - u0) + c (y2 - u0) for the first three terms
    K_EST = 8,          // Sommeijer estimate of u^{n+1} = y1 against u^n = u0, R0 = r0
    K_RKL2_PAIR = 9,    // two K_RKL2 stages j, j + 1 in one pass: out = Y_j, out2 = Y_{j+1}
    K_RKL2_RC = 10      // K_RKL2 with R0 recomputed from u0 read as a stencil (3D): the
                        // first stage's R0 (a2 = its mut_1 dt) instead of reading r0
};

// Uniform per-simulation constants the stage kernels read: passed by value as
// kernel arguments so that they live in scalar registers.
template <typename T>
struct KConsts {
    int nx, ny, nz, with_c, n_types, uniform;
    int walls, cfix;  // boundaries as in DevParams
    long long V;
    T idx2;
    T c0[NMAX], ik[NMAX], Dk[NMAX], hik[NMAX], k2[NMAX];
    T cbc[6];
};

constexpr int FMAX = NMAX + 1;  // fields of a state vector: N phases + c

template <typename T>
struct StageArgs {
    KConsts<T> K;
    const DevParams<T> *P;  // pair tables (staged into LDS by each block)
    const T *y1;    // stencil input
    const T *y2;
    const T *u0;
    const T *r0;
    T *out;
    T *out2;
    // Buffer addressing of the six vectors above: the N + 1 field planes of a
    // vector are split into ng groups (1, 2 or 4) of GS = ceil((N + 1) / ng)
    // consecutive planes whose span fits a 32-bit byte range; gb[v][g] is the
    // first plane of group g of vector v (y1, y2, u0, r0, out, out2).  Field f
    // is read from group f / GS at scalar offset (f mod GS) * plane_bytes plus a
    // 32-bit per-lane offset; kernels are compiled per ng, so both are
    // constants.
    const T *gb[6][4];
    int ng;
    unsigned plane_bytes;
    double *red;    // per-block partial sums (EST)
    long long *redn;
    // Sparse phase storage (n_p > 0): the state vectors (y1, y2, u0 and, except
    // for the RHS kind, out) hold c in plane 0, up to n_p nonzero phase values
    // in planes 1..n_p and, ids_off bytes past their base, one 32-bit word of
    // nibble phase ids per cell; r0 and out2 stay dense.  cut (may be null)
    // counts the cells the storage rule cut.
    int n_p;
    unsigned long long ids_off;
    unsigned long long *cut;
    int kind;
    T a, b, c, d, e, f;
    T a2, b2, c2, d2, e2, f2;  // K_RKL2_PAIR: coefficients of the second stage; K_RKL2_RC: a2
    // estimator
    T r_phi, a_phi, r_c, a_c, dt6, hdt;
    // tiling
    int tx, ty;      // tile of tx columns and ty rows (tile_rows(dim, N)), one block of 256 threads
    int zchunk;      // z planes per block (3D)
    int ntx, nty, nzc;
    int ntiles;
};

// Planes per buffer group for N order parameters (+ c) split into ng groups.
constexpr int group_planes(int n, int ng) { return (n + 1 + ng - 1) / ng; }

// Sparse phase storage: at most SPMAX slots per cell (their ids are the
// nibbles of one 32-bit word, 15 marking an empty slot); the value planes of
// a sparse vector are grouped as those of a dense vector of SPMAX phases.
constexpr int SPMAX = 8;
constexpr unsigned SP_EMPTY = 15u;

// The smallest group count (1, 2 or 4) whose groups span at most 2^32 - 1
// bytes for planes of V values of esz bytes, or 0 when even four do not.
inline int field_groups_needed(int n, long long V, int esz) {
    const unsigned long long pb = (unsigned long long)V * esz;
    for (int ng = 1; ng <= 4; ng *= 2)
        if ((unsigned long long)group_planes(n, ng) * pb <= 0xFFFFFFFFull) return ng;
    return 0;
}

// Fills the buffer-group bases of a StageArgs from its vector pointers, with
// at least ng_min groups (1, 2 or 4; more groups than the size needs address
// the same planes through more descriptors).  The caller guarantees
// field_groups_needed(n, V, sizeof(T)) > 0.  sparse_mask: bit v marks vector
// v (y1, y2, u0, r0, out, out2) as held in sparse storage, whose planes are
// grouped as those of SPMAX phases.
template <typename T>
inline void set_field_bases(StageArgs<T> &A, int n, long long V, int ng_min = 1,
                            unsigned sparse_mask = 0) {
    int ng = field_groups_needed(n, V, (int)sizeof(T));
    if (sparse_mask && field_groups_needed(SPMAX, V, (int)sizeof(T)) > ng)
        ng = field_groups_needed(SPMAX, V, (int)sizeof(T));
    if (ng < ng_min) ng = ng_min;
    A.ng = ng;
    A.plane_bytes = (unsigned)((unsigned long long)V * sizeof(T));
    const T *vec[6] = {A.y1, A.y2, A.u0, A.r0, A.out, A.out2};
    for (int v = 0; v < 6; ++v) {
        const int GS = group_planes((sparse_mask >> v) & 1u ? SPMAX : n, ng);
        for (int g = 0; g < 4; ++g)
            A.gb[v][g] = (vec[v] && g < ng) ? vec[v] + (long long)g * GS * V : vec[v];
    }
}

// One instance of a batch of independent 2D simulations that share N, the
// precision and with_c.
template <typename T>
struct BatchInst {
    long long off;     // element offset of the instance's state in each batch buffer
    int ntx, nty;      // tiles of the instance
    int tile0;         // first global tile of the instance
    int nsteps;        // steps of the current run (the last one possibly clipped)
    int nfull;         // steps of size dt; step nfull (if < nsteps) uses dt_last
    int s_full, s_last;  // RKL stage counts of a full and of the clipped step
    T dt, dt_last;
    T dt6, hdt;        // 6 dt and dt / 2 of the step (error estimate), rounded from double
};

// Stage-fusion depth 2 of the batched forward-Euler kernel: a tile computes
// two steps in one pass from its input with a two-cell halo.  Its LDS holds
// the input region (TILE_X + 4) x (tile rows + 4) and the first step on
// (TILE_X + 2) x (tile rows + 2), N + 3 planes each (phi, mu, Mc, c), plus the
// pair and per-phase tables; it must fit one workgroup's 64 KiB.  Depth 2 is
// built for few-field instances only (N <= DEPTH2_MAX_N): a thread holds
// N + 1 values of up to three region cells at once, which above that leaves
// one wave per SIMD.
constexpr int F2_IN_X = TILE_X + 4, F2_MID_X = TILE_X + 2;
constexpr int f2_in(int n) { return F2_IN_X * (tile_rows(2, n) + 4); }
constexpr int f2_mid(int n) { return F2_MID_X * (tile_rows(2, n) + 2); }
constexpr bool batch_depth2_fits(int esz, int n) {
    return n <= DEPTH2_MAX_N && esz * ((n + 3) * (f2_in(n) + f2_mid(n)) + 3 * n * n + 4 * n) <= 65536;
}

// Fused RKL2 stage pairs (2D): a block of P2_THREADS threads computes a tile
// of P2_TX x P2_TY cells, one per thread.  Its LDS holds the stage input with a
// two-cell halo, (P2_TX + 4) x (P2_TY + 4) cells of N + 3 planes (phi, mu, Mc,
// c), and the first stage on the tile and a one-cell ring, (P2_TX + 2) x
// (P2_TY + 2) cells of N + 2 planes (phi, mu, Mc), plus the pair and
// per-phase tables; built where that fits P2_LDS_MAX bytes.
constexpr int P2_TX = 64, P2_TY = 8, P2_THREADS = P2_TX * P2_TY, P2_LDS_MAX = 65536;
constexpr int P2_IN_X = P2_TX + 4, P2_IN_Y = P2_TY + 4, P2_IN = P2_IN_X * P2_IN_Y;
constexpr int P2_MID_X = P2_TX + 2, P2_MID_Y = P2_TY + 2, P2_MID = P2_MID_X * P2_MID_Y;
constexpr int P2_RING = P2_MID - P2_TX * P2_TY;  // cells of the one-cell ring
static_assert(P2_RING <= P2_THREADS, "one ring cell per thread");
constexpr bool rkl2_pair_fits(int esz, int n) {
    return esz * ((n + 3) * P2_IN + (n + 2) * P2_MID + 3 * n * n + 4 * n) <= P2_LDS_MAX;
}

// Fused RKL2 stage pairs (3D): a block of P3_THREADS threads marches a tile of
// P3_TX x P3_TY cells through a z extent.  Thread i owns one column of the
// tile's two-cell halo region (P3_IX x P3_IY columns): the first P3_T threads
// the tile, the next P3_M - P3_T the one-cell ring, the rest the outer ring.
// LDS holds one plane of the stage input on the halo region and one plane of
// the first stage's result on the tile and its ring, N + 2 planes each (phi,
// mu, Mc), plus the pair and per-phase tables.  Built in single precision
// for N <= P3_NMAX32 and in double precision for N <= P3_NMAX64, where the
// per-thread planes of the two z windows fit the registers of two waves per
// SIMD.
constexpr int P3_TX = 32, P3_TY = 8, P3_T = P3_TX * P3_TY;
constexpr int P3_MX = P3_TX + 2, P3_MY = P3_TY + 2, P3_M = P3_MX * P3_MY;
constexpr int P3_IX = P3_TX + 4, P3_IY = P3_TY + 4, P3_I = P3_IX * P3_IY;
constexpr int P3_THREADS = 448, P3_LDS_MAX = 65536, P3_NMAX32 = 9, P3_NMAX64 = 4;
static_assert(P3_I <= P3_THREADS && P3_THREADS % 64 == 0, "one halo-region column per thread");
// The 3D RKL2 stages that recompute R0 (K_RKL2_RC) hold the z windows of two
// stencil inputs; they are built where these fit two waves per SIMD without
// scratch: single precision N <= 9, double precision N <= 4.
constexpr bool rkl2_rc_built(int esz, int n) { return esz == 4 ? n <= 9 : n <= 4; }
constexpr bool rkl2_pair3_built(int esz, int n) {
    return (esz == 4 ? n <= P3_NMAX32 : n <= P3_NMAX64) &&
           esz * ((n + 2) * (P3_I + P3_M) + 3 * n * n + 4 * n) <= P3_LDS_MAX;
}

template <typename T>
struct BatchArgs {
    const DevParams<T> *params;  // [n]
    const BatchInst<T> *inst;    // [n]
    const int *tile_inst;        // [total_tiles] instance of each global tile
    T *bufA;                     // state at even steps
    T *bufB;                     // state at odd steps
    const int *step_base;        // device step counter (advanced by batch_tick)
    int step_offset;             // step = *step_base + step_offset
    int total_tiles;
    int depth;                   // steps per launch (stage-fusion depth): 1 or 2
    // multi-stage (RKL2) launches: stage index j of the step, the base pointers
    // of the stage's vectors by role (y1, y2, u0, r0, out, out2; null when
    // unused), the state vector (an instance's last stage writes its result
    // there), and the stage coefficients a..f per (instance, full / clipped
    // step, stage): coef[((2 i + clipped) * coef_stride + j) * 6 + 0..5]
    int kind;                    // K_EULER, K_RKL2_FIRST, K_RKL2 or K_EST
    int stage;
    const T *role[6];
    T *state;
    const T *coef;
    int coef_stride;
    // error-estimate launches (K_EST, roles y1 = u^{n+1}, u0 = u^n, r0 = R0):
    // per-tile partials at the global tile index, the norm's tolerances
    double *red;
    long long *redn;
    T r_phi, a_phi, r_c, a_c;
};

// Launchers (implemented in pf_kernels.hip).  Return hipSuccess or the launch
// error; they never synchronise.
template <typename T>
hipError_t launch_stage(int dim, int nphi, const StageArgs<T> &args, int nblocks,
                        hipStream_t stream);
template <typename T>
hipError_t launch_embed_est(const DevParams<T> *P, int nphi, int with_c, long long V,
                            const T *unew, const T *z, const T *uold, T r_phi, T a_phi, T r_c,
                            T a_c, double *red, long long *redn, int nblocks,
                            hipStream_t stream);
template <typename T>
hipError_t launch_diag(const T *u, const T *cpl, int nphi, int with_c, long long V, double *red,
                       int nblocks, hipStream_t stream);
// Conversion between dense state vectors and sparse phase storage (packing
// applies the storage rule and counts the cells it cut into *cut, if non-null).
template <typename T>
hipError_t launch_pack_sparse(const T *dense, T *sp, int nphi, int with_c, long long V, int n_p,
                              unsigned long long ids_off, unsigned long long *cut,
                              hipStream_t stream);
template <typename T>
hipError_t launch_unpack_sparse(const T *sp, T *dense, int nphi, int with_c, long long V, int n_p,
                                unsigned long long ids_off, hipStream_t stream);
hipError_t launch_finalize_norm(const double *red, const long long *redn, int nparts,
                                double *out, double seq, hipStream_t stream);
hipError_t launch_finalize_diag(const double *red, int nparts, double *out,
                                hipStream_t stream);
// Batched adaptive steps: per-instance norms from per-tile partials (ctl holds
// tile0, tile count, active flag and accept flag per instance; one block per
// instance, each in the single-instance finalisation's order) into out[3 i ..];
// the copy of out[0 .. 3 n) to host-visible memory followed by the sequence
// number seq at host_out[3 n]; the copy of each accepted instance's new state
// (len[i] elements at off[i]) from src to dst.
hipError_t launch_finalize_norm_batch(const double *red, const long long *redn, const int *ctl, int n,
                                      double *out, hipStream_t stream);
hipError_t launch_publish(const double *src, int count, double *host_out, double seq,
                          hipStream_t stream);
template <typename T>
hipError_t launch_batch_accept(const T *src, T *dst, const long long *off, const long long *len,
                               const int *ctl, int n, long long max_len, hipStream_t stream);
template <typename T>
hipError_t launch_batch_euler(int nphi, const BatchArgs<T> &args, int nblocks, hipStream_t stream);
hipError_t launch_batch_tick(int *step_base, int k, hipStream_t stream);

// Static device scratch of the allocation-free error norm: its size in bytes,
// and the device address of the current GPU's copy (looked up once per device).
constexpr size_t SCRATCH_BYTES = size_t(2) << 20;
hipError_t scratch_address(void **ptr);

bool nphi_supported(int nphi);
int supported_nphi_list(int *out, int cap);

}  // namespace pf
