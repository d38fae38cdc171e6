// pf_stage.hpp -- the fused stage kernel of the explicit phase-field +
// concentration step (gfx950).
//
// Per cell, one kernel evaluates the finite-difference right-hand side of the
// multi-phase-field equation (eq. phieq: Steinbach pairwise form, obstacle
// potential, sign as required for a stable gradient flow) and of the KKS
// concentration equation (eq. ceq in flux form, face mobility the mean of the
// two cell mobilities), forms the stage combination of the running integrator
// (Sec. 3.2: forward Euler, SSP(s)2, SSP(10)4, RKL1, RKL2) and projects the
// phi planes onto the simplex (Sec. 3.1), so that a stage is a single pass over
// HBM.  The estimator kind evaluates the Sommeijer-type local error of an
// adaptive step (Sec. 3.3) and reduces its weighted squares in FP64 per block.
//
// The path is a memory-bound stencil, so it uses no matrix cores.
//
// Decomposition.  A block is 256 threads covering a tile of the x-y plane:
// 64 x 4 cells (in 2D 64 x 8, two per thread, for N <= 4; a build option
// makes the 3D tile 32 x 8); a wavefront covers one full row of 64 cells, so
// row loads and stores are coalesced.  The tile's plane is staged in LDS
// with a one-cell halo (phi planes, chemical potential mu and mobility Mc per
// point): every thread computes mu and Mc of its own cell once, the halo
// threads those of the halo cells, and the x/y neighbours of the stencil are
// then LDS reads.  Halo and tile slots hold the periodically wrapped cells, so
// ragged tiles need no special case.  In 3D a block marches through zchunk
// planes in z and keeps planes z-1, z, z+1 of its own cell (and the halo cell
// it loads) in registers, prefetching plane z+1 while plane z is computed;
// every value is read from HBM once per march, plus the halo columns and the
// two z halo planes.  Workgroups map to tiles XCD by XCD, so that neighbouring
// tiles share one L2; in 3D the vectors other than the stencil input are
// streamed non-temporally, which keeps the stencil input's lines in L2 for the
// neighbours' halos.
//
// Addressing.  Every field plane is reached through a buffer resource of its
// vector's plane group (1, 2 or 4 groups, a compile-time parameter) and a
// 32-bit per-lane offset, so bases and descriptors stay in scalar registers.
//
// Arithmetic.  The double-precision kernels evaluate every formula in the
// oracle's order (phases ascending; neighbours x-, x+, y-, y+, z-, z+; pair
// sums over b != a) and the library is compiled without contraction, so they
// reproduce a sequential left-to-right evaluation bit for bit.  The
// single-precision kernels (the chosen form) use the same model with cheaper
// algebra: fused multiply-adds, hardware reciprocals (mu, 1/N_z, and the
// normalisation of S), per-phase sums with constants staged in LDS, the RKL
// combinations in a difference form whose weights sum to one whatever the
// rounding of the coefficients (so the total of c is kept), and, when every
// pair shares one A, B and L (a flag computed on the host), the O(N) forms
//   delta_a = A (sum_b Lap phi_b - Lap phi_a) + B (sum_b phi_b - phi_a) + psi_a
//   dphi_a/dt = L (mean of delta over the active phases - delta_a),
// which equal the pairwise sums of eq. phieq exactly in real arithmetic.
//
// The batched kernel at the end runs the same stage bodies over the tiles of
// many independent 2D simulations in one persistent launch.
#pragma once

#include <type_traits>

#include "pf_device.hpp"

namespace pf {

template <typename T>
__device__ __forceinline__ T fast_rcp(T x) {
    if constexpr (std::is_same<T, float>::value) return __builtin_amdgcn_rcpf(x);
    else return T(1) / x;
}

// IEEE maxNum (a NaN operand is ignored), so max > 0 is "some value > 0"
template <typename T>
__device__ __forceinline__ T max_num(T a, T b) {
    if constexpr (std::is_same<T, float>::value) return __builtin_fmaxf(a, b);
    else return __builtin_fmax(a, b);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    if constexpr (std::is_same<T, float>::value) return __builtin_fmaf(a, b, c);
    else return a * b + c;
}

// mu and Mc at one point (eqs. cadef, mueq, gibbs-energy, ceq).  Exact order
// for the reference (double) form; fused multiply-adds and a hardware
// reciprocal for the fast form.
// kc: per-phase constants staged in LDS (rows c0, 1/k, D/k, 1/(2k)), read by
// the fast form so that they hold no scalar registers across the z march.
template <typename T, int N, bool FAST>
__device__ __forceinline__ void point_mu_mc(const KConsts<T> &P, const T *kc, const T *v, T &mu,
                                            T &mc) {
    if constexpr (!FAST) {
        mu_mc<T, N>(P, v, mu, mc);
    } else {
        // the sums start from their first term (no added zero)
        T sc0 = v[0] * kc[0], sik = v[0] * kc[N], smc = v[0] * kc[2 * N];
#pragma unroll
        for (int a = 1; a < N; ++a) {
            sc0 = fma_t(v[a], kc[a], sc0);
            sik = fma_t(v[a], kc[N + a], sik);
            smc = fma_t(v[a], kc[2 * N + a], smc);
        }
        mu = (v[N] - sc0) * fast_rcp(sik);
        mc = smc;
    }
}

// Simplex projection S (Sec. 3.1) in the stage's arithmetic: the reference
// form divides by the sum (oracle order); the fast form multiplies by one
// hardware reciprocal of the sum instead of N divisions.
template <typename T, int N, bool FAST>
__device__ __forceinline__ void project(T *p) {
    if constexpr (!FAST) {
        simplex<T, N>(p);
    } else {
#pragma unroll
        for (int a = 0; a < N; ++a)
            if (p[a] < T(0)) p[a] = T(0);
        // the one-hot where a value reaches 1 goes to the largest value, the
        // lowest index on ties: that value is the maximum of all of them (a
        // NaN is skipped by the maximum as by the comparisons of the
        // reference form), and its first occurrence is the phase
        T pmax = p[0];
#pragma unroll
        for (int a = 1; a < N; ++a) pmax = max_num(pmax, p[a]);
        if (pmax >= T(1)) {
            bool found = false;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const bool hit = !found && p[a] == pmax;
                p[a] = hit ? T(1) : T(0);
                found = found || hit;
            }
        }
        T sum = p[0];
#pragma unroll
        for (int a = 1; a < N; ++a) sum = sum + p[a];
        if (sum > T(0)) {
            const T inv = fast_rcp(sum);
#pragma unroll
            for (int a = 0; a < N; ++a) p[a] = p[a] * inv;
        }
    }
}

// ---- sparse phase storage (Sec. 3.1 "Phase-field details") -------------------
// A state vector in sparse storage holds, per cell, c in plane 0, the values
// of its nonzero phases in slots 1..n_p (ascending phase order; empty slots
// hold 0) and a 32-bit word whose nibble s is the phase of slot s (15: empty),
// ids_off bytes past the vector's base.  Loads scatter the slots into the N
// dense values the stage arithmetic works on, so a stage in sparse storage
// computes exactly what it computes in dense storage; stores keep the nonzero
// phases.

// Id words of vector v (y1, y2, u0, r0, out, out2 by role).
template <typename T, typename S>
__device__ __forceinline__ unsigned *sparse_ids(const S &A, int v) {
    const T *b = v == 0 ? A.y1 : v == 1 ? A.y2 : v == 2 ? A.u0 : v == 3 ? A.r0 : v == 4 ? A.out : A.out2;
    return (unsigned *)((char *)const_cast<T *>(b) + A.ids_off);
}

// The N dense phase values and c of sparse vector v at byte offset boff.
template <typename T, int N, int GSS, int CP, typename S>
__device__ __forceinline__ void load_sparse(const S &A, int v, unsigned boff, bool withc, T *x) {
    const unsigned w = sparse_ids<T>(A, v)[boff / (unsigned)sizeof(T)];
    T val[SPMAX];
#pragma unroll
    for (int k = 0; k < SPMAX; ++k) val[k] = k < A.n_p ? ldv<T, GSS, CP>(A, v, k + 1, boff) : T(0);
    x[N] = withc ? ldv<T, GSS, CP>(A, v, 0, boff) : T(0);
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = T(0);
#pragma unroll
    for (int k = 0; k < SPMAX; ++k) {
        if (k < A.n_p) {  // uniform
            const unsigned id = (w >> (4 * k)) & 15u;
#pragma unroll
            for (int a = 0; a < N; ++a) x[a] = id == (unsigned)a ? val[k] : x[a];
        }
    }
}

// Stores the N dense phase values (at most n_p of them nonzero) and c into
// sparse vector v at byte offset boff.
template <typename T, int N, int GSS, int CP, typename S>
__device__ __forceinline__ void store_sparse(const S &A, int v, unsigned boff, bool withc, const T *y) {
    T slot[SPMAX];
#pragma unroll
    for (int k = 0; k < SPMAX; ++k) slot[k] = T(0);
    unsigned w = 0xFFFFFFFFu;
    // phases pushed from the highest down, so the slots end up ascending
#pragma unroll
    for (int a = N - 1; a >= 0; --a) {
        if (y[a] != T(0)) {
#pragma unroll
            for (int k = SPMAX - 1; k > 0; --k) slot[k] = slot[k - 1];
            slot[0] = y[a];
            w = (w << 4) | (unsigned)a;
        }
    }
#pragma unroll
    for (int k = 0; k < SPMAX; ++k)
        if (k < A.n_p) stv<T, GSS, CP>(A, v, k + 1, boff, slot[k]);
    if (withc) stv<T, GSS, CP>(A, v, 0, boff, y[N]);
    sparse_ids<T>(A, v)[boff / (unsigned)sizeof(T)] = w;
}

// The storage rule on a projected cell: with more than n_p nonzero phases the
// n_p largest are kept (equal values: the lower phase first), the rest set to
// 0 and the kept ones divided by their sum (the fast form multiplies by a
// hardware reciprocal).  Returns whether it cut.
template <typename T, int N, bool FAST>
__device__ __forceinline__ bool sparse_cut(T *p, int n_p) {
    int cnt = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) cnt += p[a] != T(0) ? 1 : 0;
    if (cnt <= n_p) return false;
    unsigned keep = 0u;
    for (int k = 0; k < n_p; ++k) {
        int m = -1;
        T pm = T(0);
#pragma unroll
        for (int a = 0; a < N; ++a)
            if (!((keep >> a) & 1u) && p[a] != T(0) && (m < 0 || p[a] > pm)) {
                m = a;
                pm = p[a];
            }
        keep |= 1u << m;
    }
    T sum = T(0);
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (!((keep >> a) & 1u)) p[a] = T(0);
        sum = sum + p[a];
    }
    if (sum > T(0)) {
        if constexpr (FAST) {
            const T inv = fast_rcp(sum);
#pragma unroll
            for (int a = 0; a < N; ++a) p[a] = p[a] * inv;
        } else {
#pragma unroll
            for (int a = 0; a < N; ++a) p[a] = p[a] / sum;
        }
    }
    return true;
}

// A state point of vector v: dense (GSS == 0) or in sparse storage.
template <typename T, int N, int GS, int GSS, int CP = 0, typename S>
__device__ __forceinline__ void load_state(const S &A, int v, unsigned boff, bool withc, T *x) {
    if constexpr (GSS > 0) {
        load_sparse<T, N, GSS, CP>(A, v, boff, withc, x);
    } else if constexpr (CP == 0) {
        load_point32<T, N, GS>(A, v, boff, withc, x);
    } else {
#pragma unroll
        for (int f = 0; f < N; ++f) x[f] = ldv<T, GS, CP>(A, v, f, boff);
        x[N] = withc ? ldv<T, GS, CP>(A, v, N, boff) : T(0);
    }
}

// The hardware dispatches workgroup b to XCD (b mod 8).  Each XCD gets a
// contiguous range of logical tiles (x fastest, then y, then z chunk), so tiles
// that share halo rows run on the same XCD and share its L2.  gridDim.x is a
// multiple of 8.
__device__ __forceinline__ int xcd_logical_block() {
    const int b = blockIdx.x;
    const int per = gridDim.x >> 3;
    return (b & 7) * per + (b >> 3);
}

// Debug builds (-DPF_POISON_LDS) fill an LDS region with NaN before the block
// writes it: a read of an element that no thread wrote for the current tile
// or plane then carries NaN into the results, where a comparison with the
// oracle or the non-finite count sees it.  Every thread of the block calls it
// (it ends with a barrier); in ordinary builds it is empty.
template <typename T>
__device__ __forceinline__ void poison_lds(T *p, int n) {
#ifdef PF_POISON_LDS
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = T(__builtin_nan(""));
    __syncthreads();
#else
    (void)p;
    (void)n;
#endif
}

// Pair constants A, B, L (N x N each) and the per-phase constants (rows c0,
// 1/k, D/k, 1/(2k)) of one simulation into LDS: the pairwise sums and the
// fast mu then read them without holding N^2 scalar registers.  The caller
// synchronises before they are read.
template <typename T, int N>
__device__ __forceinline__ void stage_tables(const DevParams<T> *P, T *__restrict__ pair,
                                             T *__restrict__ kc) {
    for (int i = threadIdx.x; i < 3 * N * N; i += blockDim.x) {
        const int tab = i / (N * N), ab = i % (N * N);
        const int a = ab / N, bb = ab % N;
        const T *src = tab == 0 ? P->A : tab == 1 ? P->B : P->L;
        pair[i] = src[a * NMAX + bb];
    }
    for (int i = threadIdx.x; i < 4 * N; i += blockDim.x) {
        const int row = i / N, a = i % N;
        const T *src = row == 0 ? P->c0 : row == 1 ? P->ik : row == 2 ? P->Dk : P->hik;
        kc[i] = src[a];
    }
}

// Cache policy of the operand streams of a stage (the vectors other than the
// stencil input, and the outputs): each of their values is touched once per
// stage, while the stencil input is re-read as the halo of the neighbouring
// tiles.
template <int DIM> constexpr int operand_load_cp() { return DIM == 3 ? 2 : 0; }
template <int DIM> constexpr int out_store_cp() { return DIM == 3 ? 2 : 0; }

// Operands of the stage combination at one cell: o0 from u0 (vector 2), o1
// from y2 (vector 1), o2 from r0 (vector 3), as far as the stage kind uses them.
template <typename T, int N, int KIND, int GS, int OPERAND_CP, typename S, int GSS = 0>
__device__ __forceinline__ void load_operands(const S &A, unsigned idx, bool withc, T *o0, T *o1,
                                              T *o2) {
    constexpr bool U0 = KIND == K_SSP2_FINAL || KIND == K_SSP104_S5 || KIND == K_SSP104_FINAL ||
                        KIND == K_RKL2 || KIND == K_EST;
    // the single-precision SSP(10)4 final stage is formed relative to u^n (y2)
    constexpr bool Y2 = KIND == K_RKL1 || KIND == K_RKL2 ||
                        (KIND == K_SSP104_FINAL && std::is_same<T, float>::value);
    constexpr bool R0 = KIND == K_RKL2 || KIND == K_EST;
    if constexpr (GSS > 0) {  // sparse states u0 and y2, dense R0
        if constexpr (U0) load_sparse<T, N, GSS, OPERAND_CP>(A, 2, idx, withc, o0);
        if constexpr (Y2) load_sparse<T, N, GSS, OPERAND_CP>(A, 1, idx, withc, o1);
#pragma unroll
        for (int f = 0; f <= N; ++f) {
            const bool have = f < N || withc;
            if constexpr (R0) o2[f] = have ? ldv<T, GS, OPERAND_CP>(A, 3, f, idx) : T(0);
        }
        return;
    }
#pragma unroll
    for (int f = 0; f <= N; ++f) {
        const bool have = f < N || withc;
        if constexpr (U0) o0[f] = have ? ldv<T, GS, OPERAND_CP>(A, 2, f, idx) : T(0);
        if constexpr (Y2) o1[f] = have ? ldv<T, GS, OPERAND_CP>(A, 1, f, idx) : T(0);
        if constexpr (R0) o2[f] = have ? ldv<T, GS, OPERAND_CP>(A, 3, f, idx) : T(0);
    }
}

// f(0), f(1), ..., f(R - 1) as straight-line code.  A loop, even one of a
// single trip, changes how the enclosing loop's invariants are hoisted and
// can cost the stage kernels a wavefront of occupancy.
template <int R, typename F>
__device__ __forceinline__ void unrolled(F &&f) {
    if constexpr (R > 0) {
        unrolled<R - 1>(f);
        f(R - 1);
    }
}

// v mod n.  GENERAL == false: v in [-n, 2n), by one compare each way (no
// integer division); GENERAL: any v (grids smaller than a tile).
template <bool GENERAL>
__device__ __forceinline__ int wrap_index(int v, int n) {
    if (v < 0) v += n;
    if (v >= n) v -= n;
    if constexpr (GENERAL)
        if (v < 0 || v >= n) v = (v % n + n) % n;
    return v;
}

// Whether every index a tile touches, up to two cells beyond the tiles of an
// nt-tile extent of length n (tile length t), lies in [-n, 2n) (uniform over
// the grid, so the caller branches on it once).
__device__ __forceinline__ bool wrap_fits(int nt, int t, int n) { return nt * t + 2 < 2 * n; }

// Tile L of an ntx x nty x (z chunks) tiling, x fastest.
struct TileIdx {
    int L, tix, tiy, tiz;
};
__device__ __forceinline__ TileIdx tile_index(int L, int ntx, int nty) {
    const int rest = L / ntx;
    return {L, L - rest * ntx, rest % nty, rest / nty};
}

// Index of coordinate v on an axis of n cells: wrapped on a periodic axis; on
// an axis that ends in walls, a v beyond a wall is the wall cell (zero
// gradient) and face becomes the wall's face (lo or hi) if it was unset.
// GENERAL == false: a periodic axis and v in [-n, 2n).
template <bool GENERAL>
__device__ __forceinline__ int bound_index(int v, int n, bool wall, int lo, int hi, int &face) {
    if constexpr (GENERAL) {
        if (wall) {
            if (v < 0) {
                if (face < 0) face = lo;
                return 0;
            }
            if (v >= n) {
                if (face < 0) face = hi;
                return n - 1;
            }
            return v;
        }
    }
    return wrap_index<GENERAL>(v, n);
}

// Plane offset (column) of the cell (tix * TX + lx, tiy * TY + ly), wrapped
// or held at the walls (walls: bit 0 x, bit 1 y); active: the cell lies inside
// the grid (ragged tiles); face: the wall face beyond which it lies, or -1.
template <bool GENERAL, int TX>
__device__ __forceinline__ void own_column(int tix, int tiy, int TY, int lx, int ly, int nx, int ny,
                                           int walls, long long &col, bool &active, int &face) {
    const int gx = tix * TX + lx, gy = tiy * TY + ly;
    active = gx < nx && gy < ny;
    face = -1;
    const int ix = bound_index<GENERAL>(gx, nx, walls & 1, 0, 1, face);
    const int iy = bound_index<GENERAL>(gy, ny, (walls >> 1) & 1, 2, 3, face);
    col = (long long)iy * nx + ix;
}

// Halo cell h (0 <= h < 2 TX + 2 TY) of tile (tix, tiy) of TX x TY cells:
// the edge neighbours of the tile without corners, periodically wrapped;
// hslot is its slot in an LDS plane of (TX + 2) x (TY + 2).
template <bool GENERAL, int TX>
__device__ __forceinline__ void halo_column(int tix, int tiy, int TY, int h, int nx, int ny, int walls,
                                            long long &hcol, int &hslot, int &face) {
    constexpr int TXH = TX + 2;
    int hx, hy;
    if (h < TX) { hx = h; hy = -1; }
    else if (h < 2 * TX) { hx = h - TX; hy = TY; }
    else if (h < 2 * TX + TY) { hx = -1; hy = h - 2 * TX; }
    else { hx = TX; hy = h - 2 * TX - TY; }
    hslot = (hy + 1) * TXH + (hx + 1);
    face = -1;
    const int hgx = bound_index<GENERAL>(tix * TX + hx, nx, walls & 1, 0, 1, face);
    const int hgy = bound_index<GENERAL>(tiy * TY + hy, ny, (walls >> 1) & 1, 2, 3, face);
    hcol = (long long)hgy * nx + hgx;
}

// A point loaded for a ghost cell beyond face (>= 0) that holds c fixed takes
// that c (the wall cell's phi are already its own: zero gradient).
template <typename T, int N>
__device__ __forceinline__ void fix_ghost_c(const KConsts<T> &K, int face, bool withc, T *v) {
    if (face >= 0 && withc && ((K.cfix >> face) & 1)) v[N] = K.cbc[face];
}

// Activity of the N phases at a cell: one flag per phase up to 9 phases (each
// flag stays a lane mask, so a test costs no bit extraction), a bit mask
// above (that many flags would overflow the scalar registers).
template <int N, bool FLAGS = (N <= 9)>
struct PhaseFlags {
    bool on[N];
    __device__ __forceinline__ void set(int a, bool v) { on[a] = v; }
    __device__ __forceinline__ bool operator[](int a) const { return on[a]; }
};
template <int N>
struct PhaseFlags<N, false> {
    unsigned m = 0u;
    __device__ __forceinline__ void set(int a, bool v) { m |= (v ? 1u : 0u) << a; }
    __device__ __forceinline__ bool operator[](int a) const { return (m >> a) & 1u; }
};

// Right-hand side of eqs. phieq and ceq at one cell (the per-cell part of
// every stage kind): x/y neighbours from an LDS plane tile holding the N phi
// planes, then mu, then Mc, PLANE values apart, with rows ROW apart (own: the
// cell's slot); in 3D the z neighbours come from registers (prv below, nxt
// above).  cur: the cell's own N + 1 values, mu_c / mc_c its mu and Mc.
template <typename T, int DIM, int N, bool FAST, int PLANE, int ROW>
__device__ __forceinline__ void rhs_point(const KConsts<T> &P, const T *__restrict__ lds,
                                          const T *__restrict__ pair, const T *__restrict__ kc,
                                          const int own, const T *cur, const T mu_c, const T mc_c,
                                          const T *prv, const T mu_p, const T mc_p, const T *nxt,
                                          const T mu_n, const T mc_n, T *r) {
    const bool withc = P.with_c != 0;
    const T idx2 = P.idx2;
    // activity of phase a: phi_a > 0 at the cell or at one of its 2d
    // neighbours (filter n and N_z of eq. phieq), as max > 0
    const int nbs[4] = {own - 1, own + 1, own - ROW, own + ROW};
    // the fast form starts its sums from the first term (no added zero) and
    // sums 2 Mc_face (mu_k - mu) for the flux, halved once at the end; without
    // c, mu and Mc are zero on every point, so the flux is zero unguarded
    T lap[N], mx[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        lap[a] = T(0);
        mx[a] = cur[a];
    }
    T flux = T(0);
#pragma unroll
    for (int k = 0; k < 2 * DIM; ++k) {
        T muk, mck;
        if (k < 4) {
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const T v = lds[a * PLANE + nbs[k]];
                lap[a] = (FAST && k == 0) ? v : lap[a] + v;
                mx[a] = max_num(mx[a], v);
            }
            muk = lds[N * PLANE + nbs[k]];
            mck = lds[(N + 1) * PLANE + nbs[k]];
        } else {
            const T *nv = k == 4 ? prv : nxt;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                lap[a] = lap[a] + nv[a];
                mx[a] = max_num(mx[a], nv[a]);
            }
            muk = k == 4 ? mu_p : mu_n;
            mck = k == 4 ? mc_p : mc_n;
        }
        if constexpr (FAST) {
            flux = k == 0 ? (mc_c + mck) * (muk - mu_c) : fma_t(mc_c + mck, muk - mu_c, flux);
        } else if (withc) {
            flux = flux + (T(0.5) * (mc_c + mck)) * (muk - mu_c);
        }
    }
    PhaseFlags<N> on;
    int nzc = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const bool v = mx[a] > T(0);
        on.set(a, v);
        nzc += v ? 1 : 0;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if constexpr (FAST) lap[a] = fma_t(T(-2 * DIM), cur[a], lap[a]) * idx2;
        else lap[a] = (lap[a] - T(2 * DIM) * cur[a]) * idx2;
    }

    // variational derivative delta_a = sum_{b != a} (A_ab Lap phi_b +
    // B_ab phi_b) + psi_{type(a)}(mu)
    // grand potential psi_a(mu) = -mu^2/(2k_a) - mu c0_a (Sec. 2)
    // (the fast form needs no guard: without c, mu = 0 gives psi = -0)
    T psi[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if constexpr (FAST) psi[a] = fma_t(-(mu_c * mu_c), kc[3 * N + a], -(mu_c * kc[a]));
        else if (!withc) psi[a] = T(0);
        else psi[a] = (-mu_c * mu_c) / P.k2[a] - mu_c * P.c0[a];
    }
    T delta[N];
    const T inz = FAST ? fast_rcp(T(nzc > 0 ? nzc : 1)) : T(1) / T(nzc > 0 ? nzc : 1);
    if (FAST && N == 2 && P.uniform) {
        // two phases: both active or no driving force; with both, the pair
        // form gives r_0 = L (delta_1 - delta_0) / 2 = -r_1, where
        // delta_1 - delta_0 = A (Lap phi_0 - Lap phi_1) + B (phi_0 - phi_1)
        // + psi_1 - psi_0 (the sums of the general forms, their equal terms
        // cancelled)
        const T A0 = pair[1], B0 = pair[N * N + 1], L0 = pair[2 * N * N + 1];
        const T d = fma_t(A0, lap[0] - lap[N - 1], fma_t(B0, cur[0] - cur[N - 1], psi[N - 1] - psi[0]));
        const T r0 = nzc >= 2 ? (T(0.5) * L0) * d : T(0);
        r[0] = r0;
        r[N - 1] = -r0;
    } else if (FAST && P.uniform) {
        const T A0 = pair[1], B0 = pair[N * N + 1], L0 = pair[2 * N * N + 1];
        T slap = lap[0], sp = cur[0];
#pragma unroll
        for (int a = 1; a < N; ++a) {
            slap += lap[a];
            sp += cur[a];
        }
        T dact = T(0);
#pragma unroll
        for (int a = 0; a < N; ++a) {
            const T s = fma_t(A0, slap - lap[a], B0 * (sp - cur[a])) + psi[a];
            delta[a] = s;
            if (on[a]) dact += s;
        }
        const T mean = dact * inz;
#pragma unroll
        for (int a = 0; a < N; ++a)
            r[a] = (on[a] && nzc >= 2) ? L0 * (mean - delta[a]) : T(0);
    } else {
#pragma unroll
        for (int a = 0; a < N; ++a) {
            T s = T(0);
#pragma unroll
            for (int bb = 0; bb < N; ++bb) {
                if (bb == a) continue;
                const T Aab = pair[a * N + bb], Bab = pair[N * N + a * N + bb];
                if constexpr (FAST) s = fma_t(Aab, lap[bb], fma_t(Bab, cur[bb], s));
                else s = s + (Aab * lap[bb] + Bab * cur[bb]);
            }
            if (withc) s = s + psi[a];
            delta[a] = s;
        }
        // dphi_a/dt = -(1/N_z) sum_{b active} L_ab (delta_a - delta_b)
#pragma unroll
        for (int a = 0; a < N; ++a) {
            T ra = T(0);
            if (on[a] && nzc >= 2) {
                T s = T(0);
#pragma unroll
                for (int bb = 0; bb < N; ++bb) {
                    if (bb == a || !on[bb]) continue;
                    const T Lab = pair[2 * N * N + a * N + bb];
                    if constexpr (FAST) s = fma_t(Lab, delta[a] - delta[bb], s);
                    else s = s + Lab * (delta[a] - delta[bb]);
                }
                ra = -s * inz;
            }
            r[a] = ra;
        }
    }
    if constexpr (FAST) r[N] = flux * (T(0.5) * idx2);
    else r[N] = withc ? flux * idx2 : T(0);
}

// One value of an RKL2 stage (eq. sts): (1 - mu_j - nu_j) u0 + mu_j Y_{j-1} +
// nu_j Y_{j-2} + dt (mut_j r + gam_j R0) with a = 1 - mu_j - nu_j, b = mu_j,
// c = nu_j, d = dt, e = mut_j, f = gam_j; y1 = Y_{j-1}, r = rhs(Y_{j-1}).  The
// fast form is u0 + mu_j (Y_{j-1} - u0) + nu_j (Y_{j-2} - u0), the same
// combination, whose weights sum to 1 exactly whatever the rounding of mu_j
// and nu_j (the total of c is kept).
template <typename T, bool FAST>
__device__ __forceinline__ T rkl2_value(T a, T b, T c, T d, T e, T f, T y1, T r, T u, T y2, T r0) {
    if constexpr (FAST) return fma_t(d, fma_t(e, r, f * r0), fma_t(c, y2 - u, fma_t(b, y1 - u, u)));
    else return ((a * u + b * y1) + c * y2) + d * (e * r + f * r0);
}

// The first RKL2 stage at one cell (eq. sts with the correction at the end of
// Sec. 3.2): ys = S(u^{n,0} + a r) with a = mut_1 dt and r = rhs(u^{n,0}) (cut:
// the sparse storage rule, applied after S), and r0 = R0: r, with the phi
// planes replaced by (ys - u^{n,0}) / a where S changed the cell.  The stage
// kernel that stores R0 and the stage kernel that recomputes it share this
// arithmetic, so both give the same bits.
template <typename T, int N, bool FAST, typename Cut>
__device__ __forceinline__ void rkl2_first_point(const T a, const T *cur, const T *r, T *ys, T *r0,
                                                 Cut &&cut) {
    T yv[N + 1];
#pragma unroll
    for (int f = 0; f <= N; ++f) {
        if constexpr (FAST) yv[f] = fma_t(a, r[f], cur[f]);
        else yv[f] = cur[f] + a * r[f];
        ys[f] = yv[f];
    }
    project<T, N, FAST>(ys);
    cut(ys);
    bool changed = false;
#pragma unroll
    for (int f = 0; f < N; ++f) changed = changed || bits_differ(ys[f], yv[f]);
    // (the fast form multiplies by a hardware reciprocal of mut_1 dt)
    T inv_a = T(0);
    if constexpr (FAST) inv_a = fast_rcp(a);
#pragma unroll
    for (int f = 0; f < N; ++f) {
        T ra = r[f];
        if (changed) {
            if constexpr (FAST) ra = (ys[f] - cur[f]) * inv_a;
            else ra = (ys[f] - cur[f]) / a;
        }
        r0[f] = ra;
    }
    r0[N] = r[N];
}

// Stage combination, projection and store at one cell (byte offset idx in a
// plane) from its own values cur, its right-hand side r and the operands
// o0 (u0), o1 (y2), o2 (r0) of the stage kind; the estimator kind adds its
// weighted squares to acc and its degrees of freedom to cnt.
template <typename T, int N, int KIND, int GS, int SCP, bool FAST, int GSS = 0>
__device__ __forceinline__ void cell_combine(const StageArgs<T> &A, const unsigned idx,
                                             const bool withc, const T *cur, const T *r,
                                             const T *o0, const T *o1, const T *o2, double &acc,
                                             long long &cnt) {
    // sparse storage: the storage rule after S, the state output in slots
    const auto cut = [&](T *p) __attribute__((always_inline)) {
        if constexpr (GSS > 0) {
            if (sparse_cut<T, N, FAST>(p, A.n_p) && A.cut) atomicAdd(A.cut, 1ull);
        }
    };
    const auto store_out = [&](const T *p) __attribute__((always_inline)) {
        if constexpr (GSS > 0) {
            store_sparse<T, N, GSS, SCP>(A, 4, idx, withc, p);
        } else {
#pragma unroll
            for (int f = 0; f < N; ++f) stv<T, GS, SCP>(A, 4, f, idx, p[f]);
            if (withc) stv<T, GS, SCP>(A, 4, N, idx, p[N]);
        }
    };
    T yv[N + 1];
    if constexpr (KIND == K_RHS) {
#pragma unroll
        for (int f = 0; f < N; ++f) stv<T, GS, SCP>(A, 4, f, idx, r[f]);
        if (withc) stv<T, GS, SCP>(A, 4, N, idx, r[N]);
    } else if constexpr (KIND == K_EST) {
        // e = (12 (u^n - u^{n+1}) + 6 dt (R0 + rhs(u^{n+1}))) / 15; a phi
        // entry whose trial value u^n + dt/2 (R0 + rhs(u^{n+1})) leaves
        // [0,1] has zero error; weights r max(|u^n|,|u^{n+1}|) + a; the
        // two-DoF rule for cells without nontrivial phi entries
        // (the fast form multiplies by 1/15 and by a hardware reciprocal of
        // the weight: a control quantity, where an ulp does not matter)
        const auto quot = [](T x, T y) __attribute__((always_inline)) {
            if constexpr (FAST) return x * fast_rcp(y);
            else return x / y;
        };
        const auto est = [&](T u_n, T u_1, T rs) __attribute__((always_inline)) {
            if constexpr (FAST) return (T(12) * (u_n - u_1) + A.dt6 * rs) * T(1.0 / 15.0);
            else return (T(12) * (u_n - u_1) + A.dt6 * rs) / T(15);
        };
        int nt = 0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            const T u_n = o0[a];
            const T rs = o2[a] + r[a];
            T e = est(u_n, cur[a], rs);
            const T trial = u_n + A.hdt * rs;
            if (trial < T(0) || trial > T(1)) e = T(0);
            if (e != T(0)) {
                const T w = A.r_phi * tmax(tabs(u_n), tabs(cur[a])) + A.a_phi;
                const T q = quot(e, w);
                acc += (double)q * (double)q;
                ++nt;
            }
        }
        cnt += nt > 0 ? nt : 2;
        if (withc) {
            const T u_n = o0[N];
            const T rs = o2[N] + r[N];
            const T e = est(u_n, cur[N], rs);
            const T w = A.r_c * tmax(tabs(u_n), tabs(cur[N])) + A.a_c;
            const T q = quot(e, w);
            acc += (double)q * (double)q;
            cnt += 1;
        }
    } else {
        if constexpr (KIND == K_EULER) {
            // b != 0: the sub-step of Alg. ssp2, y + dt (r / (s - 1)) with a = dt
            // and b = s - 1, in the printed order (the fast form scales r by
            // the quotient a / b in one fused multiply-add)
            if (A.b != T(0)) {
                if constexpr (FAST) {
                    const T ab = A.a / A.b;
#pragma unroll
                    for (int f = 0; f <= N; ++f) yv[f] = fma_t(ab, r[f], cur[f]);
                } else {
#pragma unroll
                    for (int f = 0; f <= N; ++f) yv[f] = cur[f] + A.a * (r[f] / A.b);
                }
            } else {
#pragma unroll
                for (int f = 0; f <= N; ++f) {
                    if constexpr (FAST) yv[f] = fma_t(A.a, r[f], cur[f]);
                    else yv[f] = cur[f] + A.a * r[f];
                }
            }
        } else if constexpr (KIND == K_SSP104_S5) {
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                if constexpr (FAST) yv[f] = fma_t(A.a, r[f], cur[f]);
                else yv[f] = cur[f] + A.a * r[f];
            }
        } else if constexpr (KIND == K_RKL2_FIRST) {
            // formed in rkl2_first_point below
        } else if constexpr (KIND == K_SSP2_FINAL) {
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                yv[f] = ((A.a * cur[f] + o0[f]) + A.b * r[f]) / A.c;
            }
        } else if constexpr (KIND == K_SSP104_FINAL) {
            // fast form, with o0 = the fifth stage value Y6' and o1 = u^n:
            // u^n + c (Y6' - u^n) + a (Y10 - u^n) + b r, the same combination
            // as q2 + a Y10 + b r, whose weights sum to one whatever the
            // rounding of a and c (the total of c is kept)
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                if constexpr (FAST)
                    yv[f] = fma_t(A.b, r[f], fma_t(A.a, cur[f] - o1[f], fma_t(A.c, o0[f] - o1[f], o1[f])));
                else
                    yv[f] = (o0[f] + A.a * cur[f]) + A.b * r[f];
            }
        } else if constexpr (KIND == K_RKL1) {
            // the fast form uses mu_j + nu_j = 1: Y_{j-1} + nu_j (Y_{j-2} -
            // Y_{j-1}), so rounded coefficients cannot change the total of c
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                if constexpr (FAST) yv[f] = fma_t(A.c, r[f], fma_t(A.b, o1[f] - cur[f], cur[f]));
                else yv[f] = (A.a * cur[f] + A.b * o1[f]) + A.c * r[f];
            }
        } else {  // K_RKL2
#pragma unroll
            for (int f = 0; f <= N; ++f)
                yv[f] = rkl2_value<T, FAST>(A.a, A.b, A.c, A.d, A.e, A.f, cur[f], r[f], o0[f], o1[f], o2[f]);
        }

        if constexpr (KIND == K_RKL2_FIRST) {
            // First RKL2 stage: Y_1 and R0 with the correction of Sec. 3.2
            T ys[N + 1], r0[N + 1];
            rkl2_first_point<T, N, FAST>(A.a, cur, r, ys, r0, cut);
            store_out(ys);
#pragma unroll
            for (int a = 0; a < N; ++a) stv<T, GS, SCP>(A, 5, a, idx, r0[a]);
            if (withc) stv<T, GS, SCP>(A, 5, N, idx, r0[N]);
        } else if constexpr (KIND == K_SSP104_S5) {
            // Fifth SSP(10)4 stage plus the two linear updates of the
            // low-storage scheme: q2 <- q2/25 + 9 q1/25, q1 <- S(15 q2 - 5 q1),
            // with q2 = u^n (o0) before them.  The fast form keeps the fifth
            // stage value Y6' itself in the q2 vector and forms
            // q1 = S(u^n + f (Y6' - u^n)), f = 2/5: the same values, with
            // weights that sum to one whatever their rounding (the final stage
            // takes the 9/25 (Y6' - u^n) part of q2).
            project<T, N, FAST>(yv);
            T q1n[N + 1];
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                const bool have = f < N || withc;
                if constexpr (FAST) {
                    if (have) stv<T, GS, SCP>(A, 5, f, idx, yv[f]);
                    q1n[f] = fma_t(A.f, yv[f] - o0[f], o0[f]);
                } else {
                    const T q2n = A.b * o0[f] + A.c * yv[f];
                    if (have) stv<T, GS, SCP>(A, 5, f, idx, q2n);
                    q1n[f] = A.d * q2n - A.e * yv[f];
                }
            }
            project<T, N, FAST>(q1n);
#pragma unroll
            for (int f = 0; f < N; ++f) stv<T, GS, SCP>(A, 4, f, idx, q1n[f]);
            if (withc) stv<T, GS, SCP>(A, 4, N, idx, q1n[N]);
        } else {
            project<T, N, FAST>(yv);
            cut(yv);
            store_out(yv);
            if constexpr (KIND == K_EULER) {
                if (A.out2 != nullptr) {
#pragma unroll
                    for (int f = 0; f < N; ++f) stv<T, GS, SCP>(A, 5, f, idx, r[f]);
                    if (withc) stv<T, GS, SCP>(A, 5, N, idx, r[N]);
                }
            }
        }
    }
}

// One tile (logical index L) of one stage.  Every thread of the block calls
// it with the same arguments (it synchronises the block).  GS: planes per
// buffer group of the vectors (see set_field_bases).  TABLES: stage the LDS
// tables of A.P first (false: the caller has staged them).  t: the tile's
// index and coordinates (tile_index, or kept by a caller that walks tiles).
// The tile is TX x TY cells, TX = tile_cols(DIM), TY = tile_rows(DIM, N);
// thread (lx, ly) = (t mod TX, t / TX) computes the R = TY / TR cells
// (lx, ly + TR k) of its column, TR = 256 / TX (3D: R = 1, marched in z).
template <typename T, int DIM, int N, int KIND, int GS, bool TABLES = true, bool WALLS = false,
          int GSS = 0>
__device__ __forceinline__ void stage_body(const StageArgs<T> &A, const TileIdx t, T *__restrict__ lds,
                                           T *__restrict__ pair, T *__restrict__ kc) {
    constexpr bool FAST = std::is_same<T, float>::value;
    constexpr int LCP = operand_load_cp<DIM>(), SCP = out_store_cp<DIM>();
    // the tile shape is fixed at compile time so that every LDS plane offset
    // is an instruction immediate; TR rows of TX threads
    constexpr int TX = tile_cols(DIM), TY = tile_rows(DIM, N), TR = thread_rows(DIM), R = TY / TR;
    constexpr int TXH = TX + 2, TYH = TY + 2;
    constexpr int plane_sz = TXH * TYH;
    static_assert(DIM == 2 || R == 1, "3D tiles march one row set in z");
    static_assert(2 * TX + 2 * TY <= 256, "one halo cell per thread");
    const KConsts<T> &P = A.K;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const bool withc = P.with_c != 0;
    const bool tile_ok = t.L < A.ntiles;  // uniform over the block

    double acc = 0.0;
    long long cnt = 0;

    if (tile_ok) {
        if constexpr (TABLES) {
            stage_tables<T, N>(A.P, pair, kc);
            __syncthreads();  // the tables are read from the first plane on
        }
        const int tix = t.tix, tiy = t.tiy, tiz = t.tiz;
        const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
        const long long nxy = (long long)nx * ny;
        // own slots hold the periodically wrapped cells (or, beyond a wall,
        // the ghost cells: the wall cell, with c fixed where the face holds it)
        int own_slot[R], own_face[R];
        long long col[R];
        bool active[R];
        const bool has_halo = threadIdx.x < 2 * TX + 2 * TY;
        long long hcol = 0;
        int hslot = 0, hface = -1;
        // walls: compiled in only for grids that have them (the periodic kernels
        // carry none of their code)
        const int walls = WALLS ? P.walls : 0;
        auto columns = [&](auto general) __attribute__((always_inline)) {
            constexpr bool G = decltype(general)::value;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                own_slot[k] = (ly + TR * k + 1) * TXH + (lx + 1);
                own_column<G, TX>(tix, tiy, TY, lx, ly + TR * k, nx, ny, walls, col[k], active[k],
                                  own_face[k]);
            }
            if (has_halo) halo_column<G, TX>(tix, tiy, TY, threadIdx.x, nx, ny, walls, hcol, hslot, hface);
        };
        if (!WALLS && wrap_fits(A.ntx, TX, nx) && wrap_fits(A.nty, TY, ny))
            columns(std::false_type{});
        else
            columns(std::true_type{});
        const bool wz = DIM == 3 && ((walls >> 2) & 1);

        const int z0 = DIM == 3 ? tiz * A.zchunk : 0;
        const int z1 = DIM == 3 ? min(z0 + A.zchunk, nz) : 1;

        T prv[N + 1], cur[R][N + 1], nxt[N + 1], hcur[N + 1], hnxt[N + 1];
        T mu_p = T(0), mc_p = T(0), mu_n = T(0), mc_n = T(0);
        T mu_c[R], mc_c[R];
        // every load of the first plane is issued before the first use of one
        if (DIM == 3) {
            const int zm = z0 == 0 ? (wz ? 0 : nz - 1) : z0 - 1;
            load_state<T, N, GS, GSS>(A, 0, (unsigned)(zm * nxy + col[0]) * (unsigned)sizeof(T), withc, prv);
        }
#pragma unroll
        for (int k = 0; k < R; ++k)
            load_state<T, N, GS, GSS>(A, 0, (unsigned)((long long)z0 * nxy + col[k]) * (unsigned)sizeof(T), withc,
                                   cur[k]);
        if (has_halo)
            load_state<T, N, GS, GSS>(A, 0, (unsigned)((long long)z0 * nxy + hcol) * (unsigned)sizeof(T), withc,
                                   hcur);
        // ghost cells that hold c fixed take it just before their first use,
        // so that the loads stay in flight; periodic grids skip all of it
        const bool ghosts = WALLS && P.cfix != 0 && withc;

        for (int z = z0; z < z1; ++z) {
            const long long pz = (long long)z * nxy;
            if (DIM == 3) {
                const int zp = z == nz - 1 ? (wz ? nz - 1 : 0) : z + 1;
                load_state<T, N, GS, GSS>(A, 0, (unsigned)((long long)zp * nxy + col[0]) * (unsigned)sizeof(T),
                                       withc, nxt);
                if (has_halo && z + 1 < z1)
                    load_state<T, N, GS, GSS>(A, 0, (unsigned)((long long)zp * nxy + hcol) * (unsigned)sizeof(T),
                                           withc, hnxt);
            }
            if (z == z0) {  // later planes rotate their mu and Mc in
                if (ghosts) {
#pragma unroll
                    for (int k = 0; k < R; ++k) fix_ghost_c<T, N>(P, own_face[k], true, cur[k]);
                    if (DIM == 3) {
                        fix_ghost_c<T, N>(P, own_face[0], true, prv);
                        if (z0 == 0 && wz) fix_ghost_c<T, N>(P, 4, true, prv);
                    }
                    if (has_halo) fix_ghost_c<T, N>(P, hface, true, hcur);
                }
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    mu_c[k] = T(0);
                    mc_c[k] = T(0);
                    if (withc) point_mu_mc<T, N, FAST>(P, kc, cur[k], mu_c[k], mc_c[k]);
                }
                if (DIM == 3 && withc) point_mu_mc<T, N, FAST>(P, kc, prv, mu_p, mc_p);
            }

            // ---- stage plane z in LDS ---------------------------------------
            poison_lds(lds, (N + 2) * plane_sz);
#pragma unroll
            for (int k = 0; k < R; ++k) {
#pragma unroll
                for (int a = 0; a < N; ++a) lds[a * plane_sz + own_slot[k]] = cur[k][a];
                lds[N * plane_sz + own_slot[k]] = mu_c[k];
                lds[(N + 1) * plane_sz + own_slot[k]] = mc_c[k];
            }
            if (has_halo) {
                T hmu = T(0), hmc = T(0);
                if (withc) point_mu_mc<T, N, FAST>(P, kc, hcur, hmu, hmc);
#pragma unroll
                for (int a = 0; a < N; ++a) lds[a * plane_sz + hslot] = hcur[a];
                lds[N * plane_sz + hslot] = hmu;
                lds[(N + 1) * plane_sz + hslot] = hmc;
            }
            if (DIM == 3 && ghosts) {
                fix_ghost_c<T, N>(P, own_face[0], true, nxt);
                if (z == nz - 1 && wz) fix_ghost_c<T, N>(P, 5, true, nxt);
            }
            if (DIM == 3 && withc) point_mu_mc<T, N, FAST>(P, kc, nxt, mu_n, mc_n);
            __syncthreads();

            unrolled<R>([&](const int k) __attribute__((always_inline)) {
                if (!active[k]) return;
                const unsigned idx = (unsigned)(pz + col[k]) * (unsigned)sizeof(T);  // byte offset
                // ---- right-hand side at the cell --------------------------------
                T r[N + 1];
                rhs_point<T, DIM, N, FAST, plane_sz, TXH>(P, lds, pair, kc, own_slot[k], cur[k], mu_c[k], mc_c[k],
                                                          prv, mu_p, mc_p, nxt, mu_n, mc_n, r);
                // ---- stage combination, projection, store -----------------------
                T o0[N + 1], o1[N + 1], o2[N + 1];
                load_operands<T, N, KIND, GS, LCP, StageArgs<T>, GSS>(A, idx, withc, o0, o1, o2);
                cell_combine<T, N, KIND, GS, SCP, FAST, GSS>(A, idx, withc, cur[k], r, o0, o1, o2, acc, cnt);
            });
            __syncthreads();  // plane z of LDS is read; the next plane may overwrite it

            if (DIM == 3) {
#pragma unroll
                for (int f = 0; f <= N; ++f) {
                    prv[f] = cur[0][f];
                    cur[0][f] = nxt[f];
                    hcur[f] = hnxt[f];
                }
                if (ghosts && has_halo) fix_ghost_c<T, N>(P, hface, true, hcur);
                mu_p = mu_c[0]; mc_p = mc_c[0];
                mu_c[0] = mu_n; mc_c[0] = mc_n;
            }
        }
    }

    if constexpr (KIND == K_EST) {
        block_sum(acc, cnt);
        if (threadIdx.x == 0 && tile_ok) {
            A.red[t.L] = acc;
            A.redn[t.L] = cnt;
        }
    }
}

// LDS per block: (N + 2) planes of (TILE_X + 2) x (tile rows + 2) values.
template <typename T, int N, int DIM>
constexpr int lds_elems() { return (N + 2) * (tile_cols(DIM) + 2) * (tile_rows(DIM, N) + 2); }

// Occupancy hint: the single-precision 3D kernels with up to 9 order
// parameters fit three wavefronts per SIMD (<= 168 VGPRs) without scratch;
// larger instances keep the compiler's choice.
constexpr int MIN_WAVES_2D = 1;
template <typename T, int DIM, int N>
constexpr int min_waves_per_eu() {
    return DIM == 2 ? MIN_WAVES_2D : (std::is_same<T, float>::value && N <= 9) ? 3 : 1;
}

// One named kernel per stage kind, so that profiles separate them; NG is the
// number of buffer groups of the vectors (1, 2 or 4).
#define PF_STAGE_KERNEL(name, kind)                                                         \
    template <typename T, int DIM, int N, int NG, bool WALLS, bool SPARSE = false>         \
    __global__ void __launch_bounds__(256)                                                 \
        __attribute__((amdgpu_waves_per_eu(min_waves_per_eu<T, DIM, N>(), 8)))             \
        name(const StageArgs<T> A) {                                                       \
        __shared__ T lds[lds_elems<T, N, DIM>()];                                          \
        __shared__ T pair[3 * N * N];                                                      \
        __shared__ T kc[4 * N];                                                            \
        poison_lds(pair, 3 * N * N);                                                       \
        poison_lds(kc, 4 * N);                                                             \
        stage_body<T, DIM, N, kind, group_planes(N, NG), true, WALLS,                      \
                   SPARSE ? group_planes(SPMAX, NG) : 0>(                                  \
            A, tile_index(xcd_logical_block(), A.ntx, A.nty), lds, pair, kc);              \
    }
PF_STAGE_KERNEL(rhs_kernel, K_RHS)
PF_STAGE_KERNEL(euler_stage_kernel, K_EULER)
PF_STAGE_KERNEL(ssp2_final_kernel, K_SSP2_FINAL)
PF_STAGE_KERNEL(ssp104_s5_kernel, K_SSP104_S5)
PF_STAGE_KERNEL(ssp104_final_kernel, K_SSP104_FINAL)
PF_STAGE_KERNEL(rkl1_stage_kernel, K_RKL1)
PF_STAGE_KERNEL(rkl2_first_stage_kernel, K_RKL2_FIRST)
PF_STAGE_KERNEL(rkl2_stage_kernel, K_RKL2)
PF_STAGE_KERNEL(estimator_kernel, K_EST)
#undef PF_STAGE_KERNEL

// One RKL2 stage j >= 2 of a periodic 3D grid (eq. sts) that recomputes R0
// instead of reading it.  u^{n,0} is read as a second stencil input, staged in
// LDS beside Y_{j-1}, and at each cell R0 = rhs(u^{n,0}) with the correction
// of the first stage (rkl2_first_point with a = A.a2 = mut_1 dt) is formed
// before the stage combination.  Four vectors move per cell-stage (Y_{j-1}
// and u^{n,0} with their halos, Y_{j-2}, Y_j) instead of five, for a second
// right-hand side per cell.  Every value is computed with the arithmetic of
// the first-stage kernel that stored R0 and of rkl2_stage_kernel, so the
// stage gives the same bits as that kernel reading the stored R0.  Dense
// storage; A.y1 = Y_{j-1}, A.y2 = Y_{j-2}, A.u0 = u^{n,0}, A.out = Y_j.  The two
// z windows need two waves per SIMD (up to 256 VGPRs): at three, 168 VGPRs
// spill to scratch.
template <typename T, int N, int NG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
    rkl2_rc_stage_kernel(const StageArgs<T> A) {
    constexpr bool FAST = std::is_same<T, float>::value;
    constexpr int GS = group_planes(N, NG);
    constexpr int LCP = operand_load_cp<3>(), SCP = out_store_cp<3>();
    constexpr int TX = tile_cols(3), TY = tile_rows(3, N);
    constexpr int TXH = TX + 2, PS = TXH * (TY + 2);
    static_assert(TX * TY == 256 && 2 * TX + 2 * TY <= 256, "one column and one halo cell per thread");
    __shared__ T lds[2 * (N + 2) * PS];  // plane z of Y_{j-1}, then of u^{n,0}: phi, mu, Mc
    __shared__ T pair[3 * N * N];
    __shared__ T kc[4 * N];
    poison_lds(pair, 3 * N * N);
    poison_lds(kc, 4 * N);
    const TileIdx t = tile_index(xcd_logical_block(), A.ntx, A.nty);
    if (t.L >= A.ntiles) return;  // uniform over the block
    const KConsts<T> &P = A.K;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const bool withc = P.with_c != 0;
    stage_tables<T, N>(A.P, pair, kc);
    __syncthreads();  // the tables are read from the first plane on

    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const long long nxy = (long long)nx * ny;
    const int own = (ly + 1) * TXH + (lx + 1);
    long long col = 0, hcol = 0;
    bool active = false;
    int face = -1, hslot = 0, hface = -1;
    const bool has_halo = threadIdx.x < 2 * TX + 2 * TY;
    if (wrap_fits(A.ntx, TX, nx) && wrap_fits(A.nty, TY, ny)) {
        own_column<false, TX>(t.tix, t.tiy, TY, lx, ly, nx, ny, 0, col, active, face);
        if (has_halo) halo_column<false, TX>(t.tix, t.tiy, TY, threadIdx.x, nx, ny, 0, hcol, hslot, hface);
    } else {
        own_column<true, TX>(t.tix, t.tiy, TY, lx, ly, nx, ny, 0, col, active, face);
        if (has_halo) halo_column<true, TX>(t.tix, t.tiy, TY, threadIdx.x, nx, ny, 0, hcol, hslot, hface);
    }
    const auto at = [nxy](int z, long long c) __attribute__((always_inline)) {
        return (unsigned)((long long)z * nxy + c) * (unsigned)sizeof(T);
    };
    const int z0 = t.tiz * A.zchunk, z1 = min(z0 + A.zchunk, nz);

    // input i = 0: Y_{j-1} (vector 0); i = 1: u^{n,0} (vector 2)
    constexpr int VEC[2] = {0, 2};
    T prv[2][N + 1], cur[2][N + 1], nxt[2][N + 1], hcur[2][N + 1], hnxt[2][N + 1];
    T mu_p[2], mc_p[2], mu_c[2], mc_c[2], mu_n[2], mc_n[2];
    // every load of the first plane is issued before the first use of one
    const int zm = z0 == 0 ? nz - 1 : z0 - 1;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        load_point32<T, N, GS>(A, VEC[i], at(zm, col), withc, prv[i]);
        load_point32<T, N, GS>(A, VEC[i], at(z0, col), withc, cur[i]);
        if (has_halo) load_point32<T, N, GS>(A, VEC[i], at(z0, hcol), withc, hcur[i]);
    }
    for (int z = z0; z < z1; ++z) {
        const int zp = z == nz - 1 ? 0 : z + 1;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            load_point32<T, N, GS>(A, VEC[i], at(zp, col), withc, nxt[i]);
            if (has_halo && z + 1 < z1) load_point32<T, N, GS>(A, VEC[i], at(zp, hcol), withc, hnxt[i]);
        }
        if (z == z0) {  // later planes rotate their mu and Mc in
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                mu_c[i] = mc_c[i] = mu_p[i] = mc_p[i] = T(0);
                if (withc) {
                    point_mu_mc<T, N, FAST>(P, kc, cur[i], mu_c[i], mc_c[i]);
                    point_mu_mc<T, N, FAST>(P, kc, prv[i], mu_p[i], mc_p[i]);
                }
            }
        }

        // ---- stage plane z of both inputs in LDS --------------------------
        poison_lds(lds, 2 * (N + 2) * PS);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            T *const l = lds + i * (N + 2) * PS;
#pragma unroll
            for (int a = 0; a < N; ++a) l[a * PS + own] = cur[i][a];
            l[N * PS + own] = mu_c[i];
            l[(N + 1) * PS + own] = mc_c[i];
            if (has_halo) {
                T hmu = T(0), hmc = T(0);
                if (withc) point_mu_mc<T, N, FAST>(P, kc, hcur[i], hmu, hmc);
#pragma unroll
                for (int a = 0; a < N; ++a) l[a * PS + hslot] = hcur[i][a];
                l[N * PS + hslot] = hmu;
                l[(N + 1) * PS + hslot] = hmc;
            }
            mu_n[i] = mc_n[i] = T(0);
            if (withc) point_mu_mc<T, N, FAST>(P, kc, nxt[i], mu_n[i], mc_n[i]);
        }
        __syncthreads();

        if (active) {
            const unsigned idx = at(z, col);
            T y2[N + 1];
#pragma unroll
            for (int f = 0; f <= N; ++f) y2[f] = (f < N || withc) ? ldv<T, GS, LCP>(A, 1, f, idx) : T(0);
            // R0 = rhs(u^{n,0}) with the first stage's correction, then the stage
            T q[N + 1], ys[N + 1], r0[N + 1];
            rhs_point<T, 3, N, FAST, PS, TXH>(P, lds + (N + 2) * PS, pair, kc, own, cur[1], mu_c[1], mc_c[1],
                                              prv[1], mu_p[1], mc_p[1], nxt[1], mu_n[1], mc_n[1], q);
            rkl2_first_point<T, N, FAST>(A.a2, cur[1], q, ys, r0, [](T *) {});
            T r[N + 1];
            rhs_point<T, 3, N, FAST, PS, TXH>(P, lds, pair, kc, own, cur[0], mu_c[0], mc_c[0], prv[0], mu_p[0],
                                              mc_p[0], nxt[0], mu_n[0], mc_n[0], r);
            double acc = 0.0;
            long long cnt = 0;
            cell_combine<T, N, K_RKL2, GS, SCP, FAST>(A, idx, withc, cur[0], r, cur[1], y2, r0, acc, cnt);
        }
        __syncthreads();  // plane z of LDS is read; the next plane may overwrite it

#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                prv[i][f] = cur[i][f];
                cur[i][f] = nxt[i][f];
                hcur[i][f] = hnxt[i][f];
            }
            mu_p[i] = mu_c[i];
            mc_p[i] = mc_c[i];
            mu_c[i] = mu_n[i];
            mc_c[i] = mc_n[i];
        }
    }
}

// One RKL2 stage value at a 2D cell whose neighbourhood is in an LDS plane
// tile (N phi planes, mu, Mc; PLANE values apart, rows ROW apart): the same
// arithmetic as the single-stage kernel's K_RKL2 path.  cur: the cell's
// Y_{j-1}; y2, u, r0: its Y_{j-2}, u0 and R0; cf: a..f of the stage.
template <typename T, int N, bool FAST, int PLANE, int ROW>
__device__ __forceinline__ void rkl2_point(const KConsts<T> &P, const T *__restrict__ lds,
                                           const T *__restrict__ pair, const T *__restrict__ kc,
                                           const int slot, const T *cur, const T *y2, const T *u,
                                           const T *r0, const T (&cf)[6], T *y) {
    T r[N + 1];
    rhs_point<T, 2, N, FAST, PLANE, ROW>(P, lds, pair, kc, slot, cur, lds[N * PLANE + slot],
                                         lds[(N + 1) * PLANE + slot], nullptr, T(0), T(0), nullptr,
                                         T(0), T(0), r);
#pragma unroll
    for (int f = 0; f <= N; ++f)
        y[f] = rkl2_value<T, FAST>(cf[0], cf[1], cf[2], cf[3], cf[4], cf[5], cur[f], r[f], u[f], y2[f], r0[f]);
    project<T, N, FAST>(y);
}

// Two consecutive RKL2 inner stages j and j + 1 (eq. sts) of one 2D tile of
// P2_TX x P2_TY cells in one pass over memory.  Stage j needs Y_{j-1} on the
// five-point stencil and Y_{j-2}, u0, R0 at the cell; stage j + 1 needs Y_j on
// the stencil and Y_{j-1}, u0, R0 at the cell.  The block stages Y_{j-1} with a
// two-cell halo (periodically wrapped) in LDS with its mu and Mc, computes Y_j
// on the tile (stored) and on a one-cell ring around it (LDS only), then
// Y_{j+1} on the tile.  Per cell that is four vectors read and two written for
// two stages, against five per stage one at a time.  Every value is computed
// with the single-stage kernel's arithmetic, so the results equal two single
// stages bit for bit.  Vectors: y1 = Y_{j-1}, y2 = Y_{j-2}, u0, r0 = R0, out =
// Y_j, out2 = Y_{j+1}, one buffer group each; coefficients a..f of stage j and
// a2..f2 of stage j + 1.  Thread i computes tile cell (i mod P2_TX, i / P2_TX) in
// both stages and, for i < P2_RING, one ring cell of stage j.
template <typename T, int N>
__device__ __forceinline__ void rkl2_pair_tile(const StageArgs<T> &A, const TileIdx t, T *__restrict__ in,
                                               T *__restrict__ mid, T *__restrict__ pair,
                                               T *__restrict__ kc) {
    constexpr bool FAST = std::is_same<T, float>::value;
    constexpr int GS = N + 1;
    constexpr int NP0 = (P2_IN + P2_THREADS - 1) / P2_THREADS;
    const KConsts<T> &P = A.K;
    const int nx = P.nx, ny = P.ny;
    const bool withc = P.with_c != 0;
    const int tid = threadIdx.x;
    const int lx = tid % P2_TX, ly = tid / P2_TX;
    const int x0 = t.tix * P2_TX - 2, y0 = t.tiy * P2_TY - 2;  // corner of the input region
    // the thread's ring cell (qx, qy) of the middle region: its top row, its
    // bottom row, then its left and right columns
    const bool ring = tid < P2_RING;
    int qx = 0, qy = 0;
    if (tid < 2 * P2_MID_X) {
        qx = tid < P2_MID_X ? tid : tid - P2_MID_X;
        qy = tid < P2_MID_X ? 0 : P2_MID_Y - 1;
    } else if (ring) {
        const int i = tid - 2 * P2_MID_X;
        qx = i < P2_TY ? 0 : P2_MID_X - 1;
        qy = 1 + (i < P2_TY ? i : i - P2_TY);
    }
    // byte offsets (one plane) of the thread's input-region points, its tile
    // cell and its ring cell, periodically wrapped
    unsigned ioff[NP0], coff = 0, roff = 0;
    auto offsets = [&](auto general) __attribute__((always_inline)) {
        constexpr bool G = decltype(general)::value;
        const auto at = [&](int px, int py) __attribute__((always_inline)) {
            return (unsigned)(wrap_index<G>(y0 + py, ny) * nx + wrap_index<G>(x0 + px, nx)) *
                   (unsigned)sizeof(T);
        };
#pragma unroll
        for (int k = 0; k < NP0; ++k) {
            const int p = tid + P2_THREADS * k;
            ioff[k] = p < P2_IN ? at(p % P2_IN_X, p / P2_IN_X) : 0u;
        }
        coff = at(lx + 2, ly + 2);
        roff = at(qx + 1, qy + 1);
    };
    if (wrap_fits(A.ntx, P2_TX, nx) && wrap_fits(A.nty, P2_TY, ny))
        offsets(std::false_type{});
    else
        offsets(std::true_type{});

    // every load of the input region is issued before the first use of one
    T v[NP0][N + 1];
#pragma unroll
    for (int k = 0; k < NP0; ++k)
        if (tid + P2_THREADS * k < P2_IN) load_point32<T, N, GS>(A, 0, ioff[k], withc, v[k]);
    stage_tables<T, N>(A.P, pair, kc);
    __syncthreads();  // the tables are read from here on
#pragma unroll
    for (int k = 0; k < NP0; ++k) {
        const int p = tid + P2_THREADS * k;
        if (p < P2_IN) {
            T mu = T(0), mc = T(0);
            if (withc) point_mu_mc<T, N, FAST>(P, kc, v[k], mu, mc);
#pragma unroll
            for (int a = 0; a < N; ++a) in[a * P2_IN + p] = v[k][a];
            in[N * P2_IN + p] = mu;
            in[(N + 1) * P2_IN + p] = mc;
            in[(N + 2) * P2_IN + p] = v[k][N];
        }
    }
    // the tile cell's operands, in flight across the barrier and the
    // right-hand side of stage j
    T u[N + 1], y2[N + 1], q0[N + 1];
    load_operands<T, N, K_RKL2, GS, 0>(A, coff, withc, u, y2, q0);
    __syncthreads();

    const T cf1[6] = {A.a, A.b, A.c, A.d, A.e, A.f};
    const T cf2[6] = {A.a2, A.b2, A.c2, A.d2, A.e2, A.f2};
    const int gx = t.tix * P2_TX + lx, gy = t.tiy * P2_TY + ly;
    const bool inside = gx < nx && gy < ny;
    auto to_mid = [&](const int q, const T *y) __attribute__((always_inline)) {
        T mu = T(0), mc = T(0);
        if (withc) point_mu_mc<T, N, FAST>(P, kc, y, mu, mc);
#pragma unroll
        for (int a = 0; a < N; ++a) mid[a * P2_MID + q] = y[a];
        mid[N * P2_MID + q] = mu;
        mid[(N + 1) * P2_MID + q] = mc;
    };

    // stage j on the tile cell: stored and put in LDS (its c is kept for
    // stage j + 1, its phi are read back from LDS)
    const int si = (ly + 2) * P2_IN_X + (lx + 2), sm = (ly + 1) * P2_MID_X + (lx + 1);
    auto in_point = [&](const int q, T *y) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < N; ++a) y[a] = in[a * P2_IN + q];
        y[N] = in[(N + 2) * P2_IN + q];
    };
    T yj_c;
    {
        T ym[N + 1], yj[N + 1];
        in_point(si, ym);
        rkl2_point<T, N, FAST, P2_IN, P2_IN_X>(P, in, pair, kc, si, ym, y2, u, q0, cf1, yj);
        if (inside) {
#pragma unroll
            for (int f = 0; f < N; ++f) stv<T, GS>(A, 4, f, coff, yj[f]);
            if (withc) stv<T, GS>(A, 4, N, coff, yj[N]);
        }
        to_mid(sm, yj);
        yj_c = yj[N];
    }
    // stage j on the ring cell (LDS only)
    if (ring) {
        T rc[N + 1], ru[N + 1], ry2[N + 1], rq0[N + 1], ry[N + 1];
        load_operands<T, N, K_RKL2, GS, 0>(A, roff, withc, ru, ry2, rq0);
        const int sr = (qy + 1) * P2_IN_X + (qx + 1);
        in_point(sr, rc);
        rkl2_point<T, N, FAST, P2_IN, P2_IN_X>(P, in, pair, kc, sr, rc, ry2, ru, rq0, cf1, ry);
        to_mid(qy * P2_MID_X + qx, ry);
    }
    __syncthreads();

    // stage j + 1 on the tile cell: Y_j on the stencil, Y_{j-1} at the cell
    T yj[N + 1], ym[N + 1], y[N + 1];
#pragma unroll
    for (int a = 0; a < N; ++a) yj[a] = mid[a * P2_MID + sm];
    yj[N] = yj_c;
    in_point(si, ym);
    rkl2_point<T, N, FAST, P2_MID, P2_MID_X>(P, mid, pair, kc, sm, yj, ym, u, q0, cf2, y);
    if (inside) {
#pragma unroll
        for (int f = 0; f < N; ++f) stv<T, GS>(A, 5, f, coff, y[f]);
        if (withc) stv<T, GS>(A, 5, N, coff, y[N]);
    }
}

// One block per tile; built where the LDS of rkl2_pair_tile fits (the launch
// refuses the others).
template <typename T, int N>
__global__ void __launch_bounds__(P2_THREADS) __attribute__((amdgpu_waves_per_eu(4, 8)))
    rkl2_pair_kernel(const StageArgs<T> A) {
    __shared__ T in[(N + 3) * P2_IN];
    __shared__ T mid[(N + 2) * P2_MID];
    __shared__ T pair[3 * N * N];
    __shared__ T kc[4 * N];
    const TileIdx t = tile_index(xcd_logical_block(), A.ntx, A.nty);
    if (t.L >= A.ntiles) return;  // uniform over the block
    poison_lds(in, (N + 3) * P2_IN);
    poison_lds(mid, (N + 2) * P2_MID);
    poison_lds(pair, 3 * N * N);
    poison_lds(kc, 4 * N);
    rkl2_pair_tile<T, N>(A, t, in, mid, pair, kc);
}

// Column of the 3D pair tile's halo region owned by thread t: (ix, iy) in
// [0, P3_IX) x [0, P3_IY), the tile at [2, P3_TX + 2) x [2, P3_TY + 2).
// Threads [0, P3_T) take the tile row by row (a wavefront covers two rows of
// P3_TX cells), [P3_T, P3_M) the one-cell ring (top row, bottom row, left and
// right columns), [P3_M, P3_I) the outer ring in the same order; the rest
// own no column (ix = iy = -1).
__device__ __forceinline__ void pair3_column(int t, int &ix, int &iy) {
    if (t < P3_T) {
        ix = 2 + t % P3_TX;
        iy = 2 + t / P3_TX;
        return;
    }
    t -= P3_T;
    if (t < 2 * P3_MX) {
        ix = 1 + (t < P3_MX ? t : t - P3_MX);
        iy = t < P3_MX ? 1 : P3_MY;
        return;
    }
    t -= 2 * P3_MX;
    if (t < 2 * P3_TY) {
        ix = t < P3_TY ? 1 : P3_MX;
        iy = 2 + (t < P3_TY ? t : t - P3_TY);
        return;
    }
    t -= 2 * P3_TY;
    if (t < 2 * P3_IX) {
        ix = t < P3_IX ? t : t - P3_IX;
        iy = t < P3_IX ? 0 : P3_IY - 1;
        return;
    }
    t -= 2 * P3_IX;
    if (t < 2 * (P3_IY - 2)) {
        ix = t < P3_IY - 2 ? 0 : P3_IX - 1;
        iy = 1 + (t < P3_IY - 2 ? t : t - (P3_IY - 2));
        return;
    }
    ix = iy = -1;
}

// Two consecutive RKL2 inner stages j and j + 1 (eq. sts) of one 3D tile
// column block in one pass over memory.  Stage j at plane k needs Y_{j-1} on
// the seven-point stencil and Y_{j-2}, u0, R0 at the cell; stage j + 1 at
// plane k - 1 needs Y_j on the stencil (its x-y neighbours on the tile's
// one-cell ring, its z neighbours at planes k - 2 and k) and Y_{j-1}, u0, R0
// at the cell.  March step k computes stage j at plane k on the tile and its
// ring, then stage j + 1 at plane k - 1 on the tile, for k from z0 - 1 to z1
// (stage j on the two planes around the extent is computed for the z
// stencil of stage j + 1 and not stored).  Each thread keeps the planes k - 1,
// k, k + 1 of Y_{j-1} at its column (and k + 2 in flight), and, on the tile,
// Y_j at planes k - 2, k - 1 and u0, R0 at plane k - 1, in registers; LDS
// holds Y_{j-1} at plane k on the halo region and Y_j at plane k - 1 on the
// tile and ring, with mu and Mc.  Per cell that is four vectors read and two
// written for two stages (plus the four z-halo planes of the extent), against
// five per stage one at a time.  Every value is computed with the
// single-stage kernel's arithmetic (rhs_point, rkl2_value, project), so the
// results equal two single stages bit for bit.  Vectors: y1 = Y_{j-1}, y2 =
// Y_{j-2}, u0, r0 = R0, out = Y_j, out2 = Y_{j+1}; coefficients a..f of stage
// j and a2..f2 of stage j + 1.  Periodic grids.
template <typename T, int N, int GS>
__device__ __forceinline__ void rkl2_pair3_tile(const StageArgs<T> &A, const TileIdx t, T *__restrict__ la,
                                                T *__restrict__ lb, T *__restrict__ pair,
                                                T *__restrict__ kc) {
    constexpr bool FAST = std::is_same<T, float>::value;
    constexpr int LCP = operand_load_cp<3>(), SCP = out_store_cp<3>();
    const KConsts<T> &P = A.K;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const bool withc = P.with_c != 0;
    const int tid = threadIdx.x;
    const bool hasI = tid < P3_I, hasM = tid < P3_M, isT = tid < P3_T;
    int ix, iy;
    pair3_column(tid, ix, iy);
    const int sI = iy * P3_IX + ix;              // slot in an LDS plane of the halo region
    const int sM = (iy - 1) * P3_MX + (ix - 1);  // slot in an LDS plane of the tile and ring
    const int gx = t.tix * P3_TX + ix - 2, gy = t.tiy * P3_TY + iy - 2;
    const bool inside = isT && gx < nx && gy < ny;
    long long col = 0;
    if (hasI) {
        if (wrap_fits(A.ntx, P3_TX, nx) && wrap_fits(A.nty, P3_TY, ny))
            col = (long long)wrap_index<false>(gy, ny) * nx + wrap_index<false>(gx, nx);
        else
            col = (long long)wrap_index<true>(gy, ny) * nx + wrap_index<true>(gx, nx);
    }
    const long long nxy = (long long)nx * ny;
    const auto zwrap = [nz](int k) __attribute__((always_inline)) {
        const int r = k % nz;
        return r < 0 ? r + nz : r;
    };
    const auto off = [&](int k) __attribute__((always_inline)) {
        return (unsigned)((long long)zwrap(k) * nxy + col) * (unsigned)sizeof(T);
    };
    const int z0 = t.tiz * A.zchunk, z1 = min(z0 + A.zchunk, nz);

    // Y_{j-1} at the column: planes z0 - 2, z0 - 1, z0 (the window of step
    // z0 - 1) and z0 + 1 in flight; every load is issued before the first use
    T prv[N + 1], cur[N + 1], nxt[N + 1], pre[N + 1];
    if (hasI) {
        load_point32<T, N, GS>(A, 0, off(z0 - 2), withc, prv);
        load_point32<T, N, GS>(A, 0, off(z0 - 1), withc, cur);
        load_point32<T, N, GS>(A, 0, off(z0), withc, nxt);
        load_point32<T, N, GS>(A, 0, off(z0 + 1), withc, pre);
    }
    stage_tables<T, N>(A.P, pair, kc);
    __syncthreads();  // the tables are read from here on
    T mup = T(0), mcp = T(0), muc = T(0), mcc = T(0), mun = T(0), mcn = T(0);
    if (hasI && withc) {
        point_mu_mc<T, N, FAST>(P, kc, prv, mup, mcp);
        point_mu_mc<T, N, FAST>(P, kc, cur, muc, mcc);
        point_mu_mc<T, N, FAST>(P, kc, nxt, mun, mcn);
    }
    // on the tile: Y_j at planes k - 2 and k - 1, u0 and R0 at plane k - 1
    T yjp[N + 1], yjc[N + 1], ku[N + 1], kr[N + 1];
    T mujp = T(0), mcjp = T(0), mujc = T(0), mcjc = T(0);
#pragma unroll
    for (int f = 0; f <= N; ++f) yjp[f] = yjc[f] = ku[f] = kr[f] = T(0);
    const T c1[6] = {A.a, A.b, A.c, A.d, A.e, A.f};
    const T c2[6] = {A.a2, A.b2, A.c2, A.d2, A.e2, A.f2};

    for (int k = z0 - 1; k <= z1; ++k) {
        const unsigned ok = off(k);
        // operands of stage j at plane k, in flight across the barrier (loading
        // them a whole march step ahead measured slower)
        T u0o[N + 1], y2o[N + 1], r0o[N + 1];
        if (hasM) load_operands<T, N, K_RKL2, GS, LCP>(A, ok, withc, u0o, y2o, r0o);
        poison_lds(la, (N + 2) * P3_I);
        if (hasI) {
#pragma unroll
            for (int a = 0; a < N; ++a) la[a * P3_I + sI] = cur[a];
            la[N * P3_I + sI] = muc;
            la[(N + 1) * P3_I + sI] = mcc;
        }
        __syncthreads();
        // stage j at plane k on the tile and its ring
        T yj[N + 1];
        T muj = T(0), mcj = T(0);
        if (hasM) {
            T r[N + 1];
            rhs_point<T, 3, N, FAST, P3_I, P3_IX>(P, la, pair, kc, sI, cur, muc, mcc, prv, mup, mcp, nxt,
                                                   mun, mcn, r);
#pragma unroll
            for (int f = 0; f <= N; ++f)
                yj[f] = rkl2_value<T, FAST>(c1[0], c1[1], c1[2], c1[3], c1[4], c1[5], cur[f], r[f], u0o[f],
                                            y2o[f], r0o[f]);
            project<T, N, FAST>(yj);
            if (withc) point_mu_mc<T, N, FAST>(P, kc, yj, muj, mcj);
            if (inside && k >= z0 && k < z1) {
#pragma unroll
                for (int f = 0; f < N; ++f) stv<T, GS, SCP>(A, 4, f, ok, yj[f]);
                if (withc) stv<T, GS, SCP>(A, 4, N, ok, yj[N]);
            }
        }
        // stage j + 1 at plane k - 1 on the tile: Y_j on the stencil (LDS holds
        // plane k - 1), Y_{j-1} (prv), u0 and R0 at the cell
        if (isT && k > z0) {
            T r[N + 1], y[N + 1];
            rhs_point<T, 3, N, FAST, P3_M, P3_MX>(P, lb, pair, kc, sM, yjc, mujc, mcjc, yjp, mujp, mcjp, yj,
                                                   muj, mcj, r);
#pragma unroll
            for (int f = 0; f <= N; ++f)
                y[f] = rkl2_value<T, FAST>(c2[0], c2[1], c2[2], c2[3], c2[4], c2[5], yjc[f], r[f], ku[f],
                                           prv[f], kr[f]);
            project<T, N, FAST>(y);
            if (inside) {
                const unsigned op = off(k - 1);
#pragma unroll
                for (int f = 0; f < N; ++f) stv<T, GS, SCP>(A, 5, f, op, y[f]);
                if (withc) stv<T, GS, SCP>(A, 5, N, op, y[N]);
            }
        }
        __syncthreads();  // both LDS planes are read; the next step may overwrite them
        poison_lds(lb, (N + 2) * P3_M);
        if (hasM) {
#pragma unroll
            for (int a = 0; a < N; ++a) lb[a * P3_M + sM] = yj[a];
            lb[N * P3_M + sM] = muj;
            lb[(N + 1) * P3_M + sM] = mcj;
        }
        if (isT) {
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                yjp[f] = yjc[f];
                yjc[f] = yj[f];
                ku[f] = u0o[f];
                kr[f] = r0o[f];
            }
            mujp = mujc; mcjp = mcjc;
            mujc = muj; mcjc = mcj;
        }
        if (hasI) {
#pragma unroll
            for (int f = 0; f <= N; ++f) {
                prv[f] = cur[f];
                cur[f] = nxt[f];
                nxt[f] = pre[f];
            }
            mup = muc; mcp = mcc;
            muc = mun; mcc = mcn;
            if (withc) point_mu_mc<T, N, FAST>(P, kc, nxt, mun, mcn);
            if (k + 3 <= z1 + 1) load_point32<T, N, GS>(A, 0, off(k + 3), withc, pre);
        }
    }
}

// One block per tile column block; built where rkl2_pair3_built (the launch
// refuses the others).
template <typename T, int N, int NG>
__global__ void __launch_bounds__(P3_THREADS) rkl2_pair3_kernel(const StageArgs<T> A) {
    __shared__ T la[(N + 2) * P3_I];
    __shared__ T lb[(N + 2) * P3_M];
    __shared__ T pair[3 * N * N];
    __shared__ T kc[4 * N];
    const TileIdx t = tile_index(xcd_logical_block(), A.ntx, A.nty);
    if (t.L >= A.ntiles) return;  // uniform over the block
    poison_lds(lb, (N + 2) * P3_M);
    poison_lds(pair, 3 * N * N);
    poison_lds(kc, 4 * N);
    rkl2_pair3_tile<T, N, group_planes(N, NG)>(A, t, la, lb, pair, kc);
}

// Stage kinds built for sparse phase storage (forward Euler, RKL1 and RKL2
// fixed steps and the RHS), periodic grids, one or two buffer groups.
template <typename T, int DIM, int N, int NG>
hipError_t launch_stage_sparse(const StageArgs<T> &A, int nblocks, hipStream_t stream) {
    if constexpr (NG > 2) {
        return hipErrorInvalidValue;
    } else {
        const dim3 grid(nblocks), block(256);
        switch (A.kind) {
        case K_RHS: hipLaunchKernelGGL((rhs_kernel<T, DIM, N, NG, false, true>), grid, block, 0, stream, A); break;
        case K_EULER: hipLaunchKernelGGL((euler_stage_kernel<T, DIM, N, NG, false, true>), grid, block, 0, stream, A); break;
        case K_RKL1: hipLaunchKernelGGL((rkl1_stage_kernel<T, DIM, N, NG, false, true>), grid, block, 0, stream, A); break;
        case K_RKL2_FIRST: hipLaunchKernelGGL((rkl2_first_stage_kernel<T, DIM, N, NG, false, true>), grid, block, 0, stream, A); break;
        case K_RKL2: hipLaunchKernelGGL((rkl2_stage_kernel<T, DIM, N, NG, false, true>), grid, block, 0, stream, A); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <typename T, int DIM, int N, int NG, bool W>
hipError_t launch_stage_dnw(const StageArgs<T> &A, int nblocks, hipStream_t stream) {
    if (A.n_p > 0) {
        if constexpr (W) return hipErrorInvalidValue;
        else return launch_stage_sparse<T, DIM, N, NG>(A, nblocks, stream);
    }
    const dim3 grid(nblocks), block(256);
    switch (A.kind) {
    case K_RHS: hipLaunchKernelGGL((rhs_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_EULER: hipLaunchKernelGGL((euler_stage_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_SSP2_FINAL: hipLaunchKernelGGL((ssp2_final_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_SSP104_S5: hipLaunchKernelGGL((ssp104_s5_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_SSP104_FINAL: hipLaunchKernelGGL((ssp104_final_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_RKL1: hipLaunchKernelGGL((rkl1_stage_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_RKL2_FIRST: hipLaunchKernelGGL((rkl2_first_stage_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_RKL2: hipLaunchKernelGGL((rkl2_stage_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_EST: hipLaunchKernelGGL((estimator_kernel<T, DIM, N, NG, W>), grid, block, 0, stream, A); break;
    case K_RKL2_RC:
        if constexpr (DIM == 3 && !W && rkl2_rc_built((int)sizeof(T), N))
            hipLaunchKernelGGL((rkl2_rc_stage_kernel<T, N, NG>), grid, block, 0, stream, A);
        else
            return hipErrorInvalidValue;
        break;
    case K_RKL2_PAIR:
        if constexpr (DIM == 2 && NG == 1 && !W && rkl2_pair_fits((int)sizeof(T), N))
            hipLaunchKernelGGL((rkl2_pair_kernel<T, N>), grid, dim3(P2_THREADS), 0, stream, A);
        else if constexpr (DIM == 3 && !W && rkl2_pair3_built((int)sizeof(T), N))
            hipLaunchKernelGGL((rkl2_pair3_kernel<T, N, NG>), grid, dim3(P3_THREADS), 0, stream, A);
        else
            return hipErrorInvalidValue;
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Grids with walls run kernels built with the wall code, for one buffer group
// only (the host admits walls on grids whose vectors fit one group).
template <typename T, int DIM, int N, int NG>
hipError_t launch_stage_dn(const StageArgs<T> &A, int nblocks, hipStream_t stream) {
    if (A.K.walls) {
        if constexpr (NG == 1) return launch_stage_dnw<T, DIM, N, NG, true>(A, nblocks, stream);
        else return hipErrorInvalidValue;
    }
    return launch_stage_dnw<T, DIM, N, NG, false>(A, nblocks, stream);
}

// One forward-Euler step at a cell whose neighbourhood is in an LDS plane
// tile (N phi planes, mu, Mc, c; PLANE values apart, rows ROW apart): the same
// arithmetic as the single-step kernel's K_EULER path.
template <typename T, int N, bool FAST, int PLANE, int ROW>
__device__ __forceinline__ void euler_point(const KConsts<T> &P, const T *__restrict__ lds,
                                            const T *__restrict__ pair, const T *__restrict__ kc,
                                            const int slot, const T dt, T *y) {
    T cur[N + 1];
#pragma unroll
    for (int a = 0; a < N; ++a) cur[a] = lds[a * PLANE + slot];
    cur[N] = lds[(N + 2) * PLANE + slot];
    T r[N + 1];
    rhs_point<T, 2, N, FAST, PLANE, ROW>(P, lds, pair, kc, slot, cur, lds[N * PLANE + slot],
                                         lds[(N + 1) * PLANE + slot], nullptr, T(0), T(0), nullptr,
                                         T(0), T(0), r);
#pragma unroll
    for (int f = 0; f <= N; ++f) {
        if constexpr (FAST) y[f] = fma_t(dt, r[f], cur[f]);
        else y[f] = cur[f] + dt * r[f];
    }
    project<T, N, FAST>(y);
}

// Two forward-Euler steps of one 2D tile in one pass (stage-fusion depth 2).
// The tile's input with a two-cell halo (periodically wrapped) is staged in
// LDS with mu and Mc; the first step is computed on the tile and a one-cell
// ring around it and kept in LDS with its mu and Mc; the second step is
// computed on the tile and stored.  Every value is computed with the
// arithmetic of the single-step kernel, so the result equals two single steps
// bit for bit.  two == false: one step (dt1) only, from the input region.
// Buffers: the state is read from A.gb[0][0] and written to A.gb[4][0] (one
// buffer group each).
template <typename T, int N>
__device__ __forceinline__ void euler2_tile(const StageArgs<T> &A, const TileIdx t, T *__restrict__ in,
                                            T *__restrict__ mid, const T *__restrict__ pair,
                                            const T *__restrict__ kc, const T dt1, const T dt2,
                                            const bool two) {
    constexpr bool FAST = std::is_same<T, float>::value;
    constexpr int SCP = out_store_cp<2>();
    const KConsts<T> &P = A.K;
    const int nx = P.nx, ny = P.ny;
    const bool withc = P.with_c != 0;
    constexpr int TY = tile_rows(2, N), R = TY / TILE_Y;  // tile height, cells per thread
    const int tix = t.tix, tiy = t.tiy;
    const int x0 = tix * TILE_X - 2, y0 = tiy * TY - 2;  // corner of the input region
    const bool fits = wrap_fits(A.ntx, TILE_X, nx) && wrap_fits(A.nty, TY, ny);

    poison_lds(in, (N + 3) * f2_in(N));
    poison_lds(mid, (N + 3) * f2_mid(N));
    // input region: every load is issued before the first use of one
    constexpr int NP0 = (f2_in(N) + 255) / 256;
    T v[NP0][N + 1];
    auto load_region = [&](auto general) __attribute__((always_inline)) {
        constexpr bool G = decltype(general)::value;
#pragma unroll
        for (int k = 0; k < NP0; ++k) {
            const int p = threadIdx.x + 256 * k;
            if (p < f2_in(N)) {
                const int px = p % F2_IN_X, py = p / F2_IN_X;
                const long long col = (long long)wrap_index<G>(y0 + py, ny) * nx + wrap_index<G>(x0 + px, nx);
                load_point32<T, N, N + 1>(A, 0, (unsigned)col * (unsigned)sizeof(T), withc, v[k]);
            }
        }
    };
    if (fits)
        load_region(std::false_type{});
    else
        load_region(std::true_type{});
#pragma unroll
    for (int k = 0; k < NP0; ++k) {
        const int p = threadIdx.x + 256 * k;
        if (p < f2_in(N)) {
            T mu = T(0), mc = T(0);
            if (withc) point_mu_mc<T, N, FAST>(P, kc, v[k], mu, mc);
#pragma unroll
            for (int a = 0; a < N; ++a) in[a * f2_in(N) + p] = v[k][a];
            in[N * f2_in(N) + p] = mu;
            in[(N + 1) * f2_in(N) + p] = mc;
            in[(N + 2) * f2_in(N) + p] = v[k][N];
        }
    }
    __syncthreads();

    // the thread's output cells (lx, ly + 4 k) of the tile
    const int lx = threadIdx.x % TILE_X, ly = threadIdx.x / TILE_X;
    T y[R][N + 1];
    if (!two) {
#pragma unroll
        for (int k = 0; k < R; ++k)
            euler_point<T, N, FAST, f2_in(N), F2_IN_X>(P, in, pair, kc,
                                                    (ly + TILE_Y * k + 2) * F2_IN_X + (lx + 2), dt1, y[k]);
    } else {
        // first step on the tile and its one-cell ring
        constexpr int NP1 = (f2_mid(N) + 255) / 256;
#pragma unroll
        for (int k = 0; k < NP1; ++k) {
            const int q = threadIdx.x + 256 * k;
            if (q < f2_mid(N)) {
                const int qx = q % F2_MID_X, qy = q / F2_MID_X;
                T w[N + 1];
                euler_point<T, N, FAST, f2_in(N), F2_IN_X>(P, in, pair, kc, (qy + 1) * F2_IN_X + (qx + 1),
                                                        dt1, w);
                T mu = T(0), mc = T(0);
                if (withc) point_mu_mc<T, N, FAST>(P, kc, w, mu, mc);
#pragma unroll
                for (int a = 0; a < N; ++a) mid[a * f2_mid(N) + q] = w[a];
                mid[N * f2_mid(N) + q] = mu;
                mid[(N + 1) * f2_mid(N) + q] = mc;
                mid[(N + 2) * f2_mid(N) + q] = w[N];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k)
            euler_point<T, N, FAST, f2_mid(N), F2_MID_X>(P, mid, pair, kc,
                                                      (ly + TILE_Y * k + 1) * F2_MID_X + (lx + 1), dt2, y[k]);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int gx = tix * TILE_X + lx, gy = tiy * TY + ly + TILE_Y * k;
        if (gx < nx && gy < ny) {
            const unsigned idx = (unsigned)((long long)gy * nx + gx) * (unsigned)sizeof(T);
#pragma unroll
            for (int f = 0; f < N; ++f) stv<T, N + 1, SCP>(A, 4, f, idx, y[k][f]);
            if (withc) stv<T, N + 1, SCP>(A, 4, N, idx, y[k][N]);
        }
    }
    __syncthreads();  // the LDS regions are read; the next tile may overwrite them
}

// LDS of the batched kernel for a fusion depth.
template <typename T, int N, int DEPTH>
constexpr int batch_lds_elems() {
    return DEPTH == 1 ? lds_elems<T, N, 2>() : (N + 3) * (f2_in(N) + f2_mid(N));
}

// Batched stages over many independent 2D instances.  A persistent grid splits
// the global tile list (tiles of all instances, one instance after the other)
// into one contiguous range per block.  A block loads an instance's constants,
// state offset and step data, and stages its LDS tables, when its walk enters
// that instance; an instance whose run (or whose step's stages) is complete is
// skipped.
// KIND == K_EULER: forward Euler, DEPTH steps per launch; launch j reads buffer
// A when j is even and B when odd (j = first step / DEPTH).
// KIND == K_RKL2_FIRST / K_RKL2: stage B.stage of one RKL2 step (eq. sts) of
// every instance, with the instance's stage count and coefficients for a full
// or for its clipped last step; the vectors come by role, and an instance's
// last stage writes the state vector.
// KIND == K_EST: the error estimate of every instance's step (Sec. 3.3) from
// the roles u^{n+1}, u^n and R0, one partial sum per tile at the tile's global
// index.
template <typename T, int N, int KIND, int DEPTH>
__global__ void __launch_bounds__(256) batch_kernel(const BatchArgs<T> B) {
    __shared__ T lds[batch_lds_elems<T, N, DEPTH>()];
    __shared__ T pair[3 * N * N];
    __shared__ T kc[4 * N];
    constexpr bool RKL = KIND == K_RKL2_FIRST || KIND == K_RKL2;
    const int step = *B.step_base + B.step_offset;
    const long long L = xcd_logical_block();
    const int g0 = (int)(L * B.total_tiles / gridDim.x);
    const int g1 = (int)((L + 1) * B.total_tiles / gridDim.x);
    if (g0 >= g1) return;
    poison_lds(pair, 3 * N * N);
    poison_lds(kc, 4 * N);
    int i = B.tile_inst[g0] - 1;
    int tile0 = 0, end = g0;  // tiles [tile0, end) belong to instance i
    StageArgs<T> A = {};
    TileIdx t = {0, 0, 0, 0};
    if constexpr (KIND == K_EST) {  // the norm's tolerances, the same for every instance
        A.r_phi = B.r_phi; A.a_phi = B.a_phi;
        A.r_c = B.r_c; A.a_c = B.a_c;
    }
    T dt2 = T(0);
    bool two = false;
    for (int g = g0; g < g1; ++g) {
        if (g >= end) {  // uniform over the block: enter instance i + 1
            ++i;
            const BatchInst<T> &I = B.inst[i];
            tile0 = I.tile0;
            end = tile0 + I.ntx * I.nty;
            const bool clipped = step >= I.nfull;
            if (step >= I.nsteps || (RKL && B.stage > (clipped ? I.s_last : I.s_full))) {
                g = end - 1;  // nothing to do for this instance
                continue;
            }
            const DevParams<T> &Q = B.params[i];
            A.K.nx = Q.nx; A.K.ny = Q.ny; A.K.nz = Q.nz;
            A.K.with_c = Q.with_c; A.K.n_types = Q.n_types; A.K.uniform = Q.uniform;
            A.K.V = Q.V; A.K.idx2 = Q.idx2;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                A.K.c0[a] = Q.c0[a]; A.K.ik[a] = Q.ik[a]; A.K.Dk[a] = Q.Dk[a];
                A.K.hik[a] = Q.hik[a]; A.K.k2[a] = Q.k2[a];
            }
            if constexpr (KIND == K_EST) {
                const T *r[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) r[v] = B.role[v] ? B.role[v] + I.off : nullptr;
                A.y1 = r[0]; A.u0 = r[2]; A.r0 = r[3];
                A.out = nullptr;
                A.gb[2][0] = A.u0;
                A.gb[3][0] = A.r0;
                A.dt6 = I.dt6;
                A.hdt = I.hdt;
                A.red = B.red + I.tile0;
                A.redn = B.redn + I.tile0;
            } else if constexpr (!RKL) {
                const bool even = ((step / DEPTH) & 1) == 0;
                A.y1 = (even ? B.bufA : B.bufB) + I.off;
                A.out = (even ? B.bufB : B.bufA) + I.off;
                A.a = step < I.nfull ? I.dt : I.dt_last;
                dt2 = step + 1 < I.nfull ? I.dt : I.dt_last;
                two = DEPTH == 2 && step + 1 < I.nsteps;
            } else {
                const int si = clipped ? I.s_last : I.s_full;
                const T *cf = B.coef + ((size_t)(2 * i + (clipped ? 1 : 0)) * B.coef_stride + B.stage) * 6;
                A.a = cf[0]; A.b = cf[1]; A.c = cf[2]; A.d = cf[3]; A.e = cf[4]; A.f = cf[5];
                const T *r[6];
#pragma unroll
                for (int v = 0; v < 6; ++v) r[v] = B.role[v] ? B.role[v] + I.off : nullptr;
                A.y1 = r[0]; A.y2 = r[1]; A.u0 = r[2]; A.r0 = r[3];
                // the step's last stage writes the instance's state (it reads the
                // state only at its own cell, as u0, before writing it)
                A.out = B.stage == si ? B.state + I.off : const_cast<T *>(r[4]);
                A.out2 = const_cast<T *>(r[5]);
                A.gb[1][0] = A.y2;
                A.gb[2][0] = A.u0;
                A.gb[3][0] = A.r0;
                A.gb[5][0] = A.out2;
            }
            // one buffer group per vector: the host admits only instances whose
            // state spans less than 4 GiB
            A.ng = 1;
            A.plane_bytes = (unsigned)(A.K.V * (long long)sizeof(T));
            A.gb[0][0] = A.y1;
            A.gb[4][0] = A.out;
            A.kind = KIND;
            A.tx = TILE_X;
            A.ty = tile_rows(2, N);
            A.zchunk = 1;
            A.ntx = I.ntx;
            A.nty = I.nty;
            A.nzc = 1;
            A.ntiles = I.ntx * I.nty;
            t = tile_index(g - tile0, A.ntx, A.nty);  // later tiles step in x, then y
            // the previous tile's last barrier follows its last table read
            stage_tables<T, N>(B.params + i, pair, kc);
            __syncthreads();
        }
        if constexpr (KIND == K_EULER && DEPTH == 2)
            euler2_tile<T, N>(A, t, lds, lds + (N + 3) * f2_in(N), pair, kc, A.a, dt2, two);
        else
            stage_body<T, 2, N, KIND, N + 1, false>(A, t, lds, pair, kc);
        ++t.L;
        if (++t.tix == A.ntx) {
            t.tix = 0;
            ++t.tiy;
        }
    }
}

template <typename T, int N>
hipError_t launch_batch_euler_n(const BatchArgs<T> &B, int nblocks, hipStream_t stream) {
    const dim3 grid(nblocks), block(256);
    if (B.kind == K_EST) {
        hipLaunchKernelGGL((batch_kernel<T, N, K_EST, 1>), grid, block, 0, stream, B);
    } else if (B.kind == K_RKL2_FIRST) {
        hipLaunchKernelGGL((batch_kernel<T, N, K_RKL2_FIRST, 1>), grid, block, 0, stream, B);
    } else if (B.kind == K_RKL2) {
        hipLaunchKernelGGL((batch_kernel<T, N, K_RKL2, 1>), grid, block, 0, stream, B);
    } else if (B.kind != K_EULER) {
        return hipErrorInvalidValue;
    } else if (B.depth == 1) {
        hipLaunchKernelGGL((batch_kernel<T, N, K_EULER, 1>), grid, block, 0, stream, B);
    } else if (B.depth == 2) {
        if constexpr (batch_depth2_fits(sizeof(T), N))
            hipLaunchKernelGGL((batch_kernel<T, N, K_EULER, 2>), grid, block, 0, stream, B);
        else
            return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int N, int NG>
hipError_t launch_stage_n(int dim, const StageArgs<T> &A, int nblocks, hipStream_t stream) {
    return dim == 3 ? launch_stage_dn<T, 3, N, NG>(A, nblocks, stream)
                    : launch_stage_dn<T, 2, N, NG>(A, nblocks, stream);
}

}  // namespace pf
