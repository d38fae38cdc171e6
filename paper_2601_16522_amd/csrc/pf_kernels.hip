// pf_kernels.hip -- gfx950 kernels of the explicit phase-field + concentration step.
//
// One fused kernel evaluates, per cell, the finite-difference right-hand side
// of the multi-phase-field equation (eq. phieq, Steinbach pairwise form with the
// obstacle potential) and of the KKS concentration equation (eq. ceq), forms
// the stage combination of the running integrator (Sec. 3.2: forward Euler,
// SSP(s)2, SSP(10)4, RKL1, RKL2) and applies the simplex projection to the phi
// planes (Sec. 3.1), so that each stage is a single pass over HBM.  The same
// kernel also evaluates the Sommeijer-type error estimate of an adaptive step
// (Sec. 3.3) and reduces it in FP64 per block.
//
// The path is a memory-bound stencil (tens of flops per byte at most), so it
// uses no matrix cores.  Work decomposition: a block is 256 threads covering a
// tile of tx x ty cells in the x-y plane (one wavefront spans 64 consecutive
// x cells, so every load and store of a plane row is coalesced).  In 3D a block
// marches through zchunk planes in z, keeping the planes z-1, z, z+1 of its own
// cells in registers, so every value is read from HBM once per march plus the
// two z halo planes; x and y neighbours come from the caches (the rows of the
// same tile are loaded by the block's other wavefronts, halo rows by the
// neighbouring tile of the same XCD, see the tile remap below).
//
// Floating-point order: every sum is accumulated in a fixed order (phases
// ascending; neighbours x-, x+, y-, y+, z-, z+) and the file is compiled
// without contraction, so the double-precision kernel reproduces a sequential
// left-to-right evaluation of the same formulas bit for bit.

#include "pf_internal.h"

namespace pf {

template <typename T>
__device__ __forceinline__ bool bits_differ(T a, T b);
template <>
__device__ __forceinline__ bool bits_differ<float>(float a, float b) {
    return __float_as_uint(a) != __float_as_uint(b);
}
template <>
__device__ __forceinline__ bool bits_differ<double>(double a, double b) {
    return __double_as_longlong(a) != __double_as_longlong(b);
}

template <typename T>
__device__ __forceinline__ T tabs(T v) { return v < T(0) ? -v : v; }
template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }

// KKS chemical potential and diffusive mobility at one point (eqs. cadef,
// mueq, gibbs-energy, ceq): mu = (c - sum phi_a c0_a) / (sum phi_a / k_a),
// Mc = sum phi_a D_a / k_a.
template <typename T, int N>
__device__ __forceinline__ void mu_mc(const DevParams<T> &P, const T *v, T &mu, T &mc) {
    T sc0 = T(0), sik = T(0), smc = T(0);
#pragma unroll
    for (int a = 0; a < N; ++a) {
        sc0 = sc0 + v[a] * P.c0[a];
        sik = sik + v[a] * P.ik[a];
        smc = smc + v[a] * P.Dk[a];
    }
    mu = (v[N] - sc0) / sik;
    mc = smc;
}

// Simplex projection S (Sec. 3.1): negatives to zero; if some entry is >= 1
// the largest (lowest index on ties) becomes 1 and the rest 0; divide by the sum.
template <typename T, int N>
__device__ __forceinline__ void simplex(T *p) {
#pragma unroll
    for (int a = 0; a < N; ++a)
        if (p[a] < T(0)) p[a] = T(0);
    int m = -1;
    T pm = T(0);
#pragma unroll
    for (int a = 0; a < N; ++a)
        if (p[a] >= T(1) && (m < 0 || p[a] > pm)) {
            m = a;
            pm = p[a];
        }
    if (m >= 0) {
#pragma unroll
        for (int a = 0; a < N; ++a) p[a] = (a == m) ? T(1) : T(0);
    }
    T s = T(0);
#pragma unroll
    for (int a = 0; a < N; ++a) s = s + p[a];
    if (s > T(0)) {
#pragma unroll
        for (int a = 0; a < N; ++a) p[a] = p[a] / s;
    }
}

template <typename T, int N>
__device__ __forceinline__ void load_point(const T *__restrict__ u, long long V, long long idx,
                                           bool withc, T *v) {
#pragma unroll
    for (int f = 0; f < N; ++f) v[f] = u[f * V + idx];
    v[N] = withc ? u[N * V + idx] : T(0);
}

// Deterministic block reduction of (sum, count) over a 256-thread block: a
// fixed shuffle tree inside each wavefront, then the four wavefront results in
// order.  Thread 0 returns the block totals.
__device__ __forceinline__ void block_sum(double &acc, long long &cnt) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_down(acc, off, 64);
        cnt += __shfl_down(cnt, off, 64);
    }
    __shared__ double sa[4];
    __shared__ long long sc[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sa[w] = acc;
        sc[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        acc = ((sa[0] + sa[1]) + sa[2]) + sa[3];
        cnt = ((sc[0] + sc[1]) + sc[2]) + sc[3];
    }
}

template <typename T, int DIM, int N>
__global__ void __launch_bounds__(256) stage_kernel(const StageArgs<T> A) {
    const DevParams<T> &P = *A.P;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const long long V = P.V;
    const bool withc = P.with_c != 0;
    const T idx2 = P.idx2;

    // The hardware dispatches workgroup b to XCD (b mod 8).  Each XCD gets a
    // contiguous range of logical tiles (x fastest, then y, then z chunk), so
    // tiles that share halo rows run on the same XCD and share its L2.
    const int b = blockIdx.x;
    const int per = gridDim.x >> 3;
    const int L = (b & 7) * per + (b >> 3);
    const bool tile_ok = L < A.ntiles;
    const int tix = L % A.ntx;
    const int rest = L / A.ntx;
    const int tiy = rest % A.nty;
    const int tiz = rest / A.nty;
    const int lx = threadIdx.x % A.tx, ly = threadIdx.x / A.tx;
    const int x = tix * A.tx + lx, y = tiy * A.ty + ly;
    const bool active = tile_ok && x < nx && y < ny;

    double acc = 0.0;
    long long cnt = 0;

    if (active) {
        const T *__restrict__ y1 = A.y1;
        const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        const long long nxy = (long long)nx * ny;
        const int z0 = DIM == 3 ? tiz * A.zchunk : 0;
        const int z1 = DIM == 3 ? min(z0 + A.zchunk, nz) : 1;

        T prv[N + 1], cur[N + 1], nxt[N + 1];
        const long long col = (long long)y * nx + x;
        if (DIM == 3) {
            const int zm = z0 == 0 ? nz - 1 : z0 - 1;
            load_point<T, N>(y1, V, zm * nxy + col, withc, prv);
        }
        load_point<T, N>(y1, V, (long long)z0 * nxy + col, withc, cur);

        for (int z = z0; z < z1; ++z) {
            const long long pz = (long long)z * nxy;
            const long long idx = pz + col;
            if (DIM == 3) {
                const int zp = z == nz - 1 ? 0 : z + 1;
                load_point<T, N>(y1, V, (long long)zp * nxy + col, withc, nxt);
            }

            // ---- right-hand side at (x, y, z) -----------------------------
            T mu0 = T(0), mc0 = T(0);
            if (withc) mu_mc<T, N>(P, cur, mu0, mc0);
            unsigned act = 0u;
            T lap[N];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                lap[a] = T(0);
                if (cur[a] > T(0)) act |= 1u << a;
            }
            T flux = T(0);
#pragma unroll
            for (int k = 0; k < 2 * DIM; ++k) {
                T nb[N + 1];
                if (k < 4) {
                    long long o;
                    if (k == 0) o = pz + (long long)y * nx + xm;
                    else if (k == 1) o = pz + (long long)y * nx + xp;
                    else if (k == 2) o = pz + (long long)ym * nx + x;
                    else o = pz + (long long)yp * nx + x;
                    load_point<T, N>(y1, V, o, withc, nb);
                } else {
#pragma unroll
                    for (int f = 0; f <= N; ++f) nb[f] = (k == 4) ? prv[f] : nxt[f];
                }
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    lap[a] = lap[a] + nb[a];
                    if (nb[a] > T(0)) act |= 1u << a;
                }
                if (withc) {
                    T muk, mck;
                    mu_mc<T, N>(P, nb, muk, mck);
                    flux = flux + (T(0.5) * (mc0 + mck)) * (muk - mu0);
                }
            }
            const int nzc = __popc(act);
#pragma unroll
            for (int a = 0; a < N; ++a) lap[a] = (lap[a] - T(2 * DIM) * cur[a]) * idx2;

            T psi[TMAX];
            if (withc) {
#pragma unroll
                for (int t = 0; t < TMAX; ++t)
                    psi[t] = (t < P.n_types) ? (-mu0 * mu0) / P.k2t[t] - mu0 * P.c0t[t] : T(0);
            }
            T delta[N];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                T s = T(0);
#pragma unroll
                for (int bb = 0; bb < N; ++bb) {
                    if (bb == a) continue;
                    s = s + (P.A[a * NMAX + bb] * lap[bb] + P.B[a * NMAX + bb] * cur[bb]);
                }
                if (withc) {
                    const int t = P.tphi[a];
                    const T ps = t == 0 ? psi[0] : t == 1 ? psi[1] : t == 2 ? psi[2] : psi[3];
                    s = s + ps;
                }
                delta[a] = s;
            }
            T r[N + 1];
            const T inz = T(1) / T(nzc > 0 ? nzc : 1);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                T ra = T(0);
                if (((act >> a) & 1u) && nzc >= 2) {
                    T s = T(0);
#pragma unroll
                    for (int bb = 0; bb < N; ++bb) {
                        if (bb == a || !((act >> bb) & 1u)) continue;
                        s = s + P.L[a * NMAX + bb] * (delta[a] - delta[bb]);
                    }
                    ra = -s * inz;
                }
                r[a] = ra;
            }
            r[N] = withc ? flux * idx2 : T(0);

            // ---- stage combination, projection, store --------------------
            const int kind = A.kind;
            T *__restrict__ out = A.out;
            T yv[N + 1];
            if (kind == K_RHS) {
#pragma unroll
                for (int f = 0; f < N; ++f) out[f * V + idx] = r[f];
                if (withc) out[N * V + idx] = r[N];
            } else if (kind == K_EST) {
                const T *__restrict__ un = A.u0;
                const T *__restrict__ r0 = A.r0;
                int nt = 0;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const T u_n = un[a * V + idx];
                    const T rs = r0[a * V + idx] + r[a];
                    T e = (T(12) * (u_n - cur[a]) + A.dt6 * rs) / T(15);
                    const T trial = u_n + A.hdt * rs;
                    if (trial < T(0) || trial > T(1)) e = T(0);
                    if (e != T(0)) {
                        const T w = A.r_phi * tmax(tabs(u_n), tabs(cur[a])) + A.a_phi;
                        const T q = e / w;
                        acc += (double)q * (double)q;
                        ++nt;
                    }
                }
                cnt += nt > 0 ? nt : 2;
                if (withc) {
                    const T u_n = un[N * V + idx];
                    const T rs = r0[N * V + idx] + r[N];
                    const T e = (T(12) * (u_n - cur[N]) + A.dt6 * rs) / T(15);
                    const T w = A.r_c * tmax(tabs(u_n), tabs(cur[N])) + A.a_c;
                    const T q = e / w;
                    acc += (double)q * (double)q;
                    cnt += 1;
                }
            } else {
                if (kind == K_EULER || kind == K_SSP104_S5 || kind == K_RKL2_FIRST) {
#pragma unroll
                    for (int f = 0; f <= N; ++f) yv[f] = cur[f] + A.a * r[f];
                } else if (kind == K_SSP2_FINAL) {
                    const T *__restrict__ u0 = A.u0;
#pragma unroll
                    for (int f = 0; f <= N; ++f) {
                        const T u = (f < N || withc) ? u0[f * V + idx] : T(0);
                        yv[f] = ((A.a * cur[f] + u) + A.b * r[f]) / A.c;
                    }
                } else if (kind == K_SSP104_FINAL) {
                    const T *__restrict__ u0 = A.u0;
#pragma unroll
                    for (int f = 0; f <= N; ++f) {
                        const T u = (f < N || withc) ? u0[f * V + idx] : T(0);
                        yv[f] = (u + A.a * cur[f]) + A.b * r[f];
                    }
                } else if (kind == K_RKL1) {
                    const T *__restrict__ y2 = A.y2;
#pragma unroll
                    for (int f = 0; f <= N; ++f) {
                        const T v2 = (f < N || withc) ? y2[f * V + idx] : T(0);
                        yv[f] = (A.a * cur[f] + A.b * v2) + A.c * r[f];
                    }
                } else {  // K_RKL2
                    const T *__restrict__ u0 = A.u0;
                    const T *__restrict__ y2 = A.y2;
                    const T *__restrict__ r0 = A.r0;
#pragma unroll
                    for (int f = 0; f <= N; ++f) {
                        const bool have = f < N || withc;
                        const T u = have ? u0[f * V + idx] : T(0);
                        const T v2 = have ? y2[f * V + idx] : T(0);
                        const T q0 = have ? r0[f * V + idx] : T(0);
                        yv[f] = ((A.a * u + A.b * cur[f]) + A.c * v2) + A.d * (A.e * r[f] + A.f * q0);
                    }
                }

                if (kind == K_RKL2_FIRST) {
                    // First RKL2 stage: where S changes the cell, replace rhs(u^{n,0})
                    // of the phi planes by (S(u^{n,1}) - u^{n,0}) / (mut_1 dt) (Sec. 3.2).
                    T ys[N];
#pragma unroll
                    for (int a = 0; a < N; ++a) ys[a] = yv[a];
                    simplex<T, N>(ys);
                    bool changed = false;
#pragma unroll
                    for (int a = 0; a < N; ++a) changed = changed || bits_differ(ys[a], yv[a]);
                    T *__restrict__ o2 = A.out2;
#pragma unroll
                    for (int a = 0; a < N; ++a) {
                        out[a * V + idx] = ys[a];
                        o2[a * V + idx] = changed ? (ys[a] - cur[a]) / A.a : r[a];
                    }
                    if (withc) {
                        out[N * V + idx] = yv[N];
                        o2[N * V + idx] = r[N];
                    }
                } else if (kind == K_SSP104_S5) {
                    // Fifth SSP(10)4 stage plus the two linear updates of the
                    // low-storage scheme: q2 <- q2/25 + 9 q1/25, q1 <- S(15 q2 - 5 q1).
                    simplex<T, N>(yv);
                    const T *__restrict__ q2 = A.u0;
                    T *__restrict__ o2 = A.out2;
                    T q1n[N + 1];
#pragma unroll
                    for (int f = 0; f <= N; ++f) {
                        const bool have = f < N || withc;
                        const T q2v = have ? q2[f * V + idx] : T(0);
                        const T q2n = A.b * q2v + A.c * yv[f];
                        if (have) o2[f * V + idx] = q2n;
                        q1n[f] = A.d * q2n - A.e * yv[f];
                    }
                    simplex<T, N>(q1n);
#pragma unroll
                    for (int f = 0; f < N; ++f) out[f * V + idx] = q1n[f];
                    if (withc) out[N * V + idx] = q1n[N];
                } else {
                    simplex<T, N>(yv);
#pragma unroll
                    for (int f = 0; f < N; ++f) out[f * V + idx] = yv[f];
                    if (withc) out[N * V + idx] = yv[N];
                    if (kind == K_EULER && A.out2 != nullptr) {
                        T *__restrict__ o2 = A.out2;
#pragma unroll
                        for (int f = 0; f < N; ++f) o2[f * V + idx] = r[f];
                        if (withc) o2[N * V + idx] = r[N];
                    }
                }
            }

            if (DIM == 3) {
#pragma unroll
                for (int f = 0; f <= N; ++f) {
                    prv[f] = cur[f];
                    cur[f] = nxt[f];
                }
            }
        }
    }

    if (A.kind == K_EST) {
        block_sum(acc, cnt);
        if (threadIdx.x == 0 && tile_ok) {
            A.red[L] = acc;
            A.redn[L] = cnt;
        }
    }
}

// Embedded-solution estimate (SSP(s)2, e = u^{n+1} - z) with the same norm
// terms; grid-stride over cells, deterministic per-block partials.
template <typename T>
__global__ void __launch_bounds__(256)
embed_kernel(const DevParams<T> *P, int nphi, int withc, long long V, const T *__restrict__ unew,
             const T *__restrict__ z, const T *__restrict__ uold, T r_phi, T a_phi, T r_c, T a_c,
             double *red, long long *redn) {
    double acc = 0.0;
    long long cnt = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
        int nt = 0;
        for (int a = 0; a < nphi; ++a) {
            const long long k = a * V + i;
            const T e = unew[k] - z[k];
            if (e != T(0)) {
                const T w = r_phi * tmax(tabs(uold[k]), tabs(unew[k])) + a_phi;
                const T q = e / w;
                acc += (double)q * (double)q;
                ++nt;
            }
        }
        cnt += nt > 0 ? nt : 2;
        if (withc) {
            const long long k = nphi * V + i;
            const T e = unew[k] - z[k];
            const T w = r_c * tmax(tabs(uold[k]), tabs(unew[k])) + a_c;
            const T q = e / w;
            acc += (double)q * (double)q;
            cnt += 1;
        }
    }
    block_sum(acc, cnt);
    if (threadIdx.x == 0) {
        red[blockIdx.x] = acc;
        redn[blockIdx.x] = cnt;
    }
}

// Constraint and conservation diagnostics: per block (sum c, max |sum phi - 1|,
// min phi, max phi, non-finite count), FP64, fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
diag_kernel(const T *__restrict__ u, int nphi, int withc, long long V, double *red) {
    double sc = 0.0, dev = 0.0, lo = 1e300, hi = -1e300, bad = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
        double s = 0.0;
        for (int a = 0; a < nphi; ++a) {
            const double p = (double)u[a * V + i];
            if (!isfinite(p)) bad += 1.0;
            s += p;
            lo = p < lo ? p : lo;
            hi = p > hi ? p : hi;
        }
        const double d = s > 1.0 ? s - 1.0 : 1.0 - s;
        dev = d > dev ? d : dev;
        if (withc) {
            const double c = (double)u[nphi * V + i];
            if (!isfinite(c)) bad += 1.0;
            sc += c;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sc += __shfl_down(sc, off, 64);
        const double d2 = __shfl_down(dev, off, 64);
        const double l2 = __shfl_down(lo, off, 64);
        const double h2 = __shfl_down(hi, off, 64);
        bad += __shfl_down(bad, off, 64);
        dev = d2 > dev ? d2 : dev;
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    __shared__ double s5[4][5];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        s5[w][0] = sc; s5[w][1] = dev; s5[w][2] = lo; s5[w][3] = hi; s5[w][4] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double o0 = s5[0][0], o1 = s5[0][1], o2 = s5[0][2], o3 = s5[0][3], o4 = s5[0][4];
        for (int k = 1; k < 4; ++k) {
            o0 += s5[k][0];
            o1 = s5[k][1] > o1 ? s5[k][1] : o1;
            o2 = s5[k][2] < o2 ? s5[k][2] : o2;
            o3 = s5[k][3] > o3 ? s5[k][3] : o3;
            o4 += s5[k][4];
        }
        double *r = red + 5 * (long long)blockIdx.x;
        r[0] = o0; r[1] = o1; r[2] = o2; r[3] = o3; r[4] = o4;
    }
}

// Final reductions: one 256-thread block, fixed strided order then the tree.
__global__ void __launch_bounds__(256)
finalize_norm_kernel(const double *red, const long long *redn, int n, double *out) {
    double acc = 0.0;
    long long cnt = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        acc += red[i];
        cnt += redn[i];
    }
    block_sum(acc, cnt);
    if (threadIdx.x == 0) {
        out[0] = acc;
        out[1] = (double)cnt;
        out[2] = cnt > 0 ? sqrt(acc / (double)cnt) : 0.0;
    }
}

__global__ void __launch_bounds__(256)
finalize_diag_kernel(const double *red, int n, double *out) {
    __shared__ double sh[256][5];
    double o0 = 0.0, o1 = 0.0, o2 = 1e300, o3 = -1e300, o4 = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double *r = red + 5 * (long long)i;
        o0 += r[0];
        o1 = r[1] > o1 ? r[1] : o1;
        o2 = r[2] < o2 ? r[2] : o2;
        o3 = r[3] > o3 ? r[3] : o3;
        o4 += r[4];
    }
    sh[threadIdx.x][0] = o0; sh[threadIdx.x][1] = o1; sh[threadIdx.x][2] = o2;
    sh[threadIdx.x][3] = o3; sh[threadIdx.x][4] = o4;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            double *a = sh[threadIdx.x], *b = sh[threadIdx.x + s];
            a[0] += b[0];
            a[1] = b[1] > a[1] ? b[1] : a[1];
            a[2] = b[2] < a[2] ? b[2] : a[2];
            a[3] = b[3] > a[3] ? b[3] : a[3];
            a[4] += b[4];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] = sh[0][k];
}

// ------------------------------------------------------------------------
// Dispatch over the compiled (dim, N) instances
// ------------------------------------------------------------------------

#define PF_NPHI_LIST(X) X(2) X(3) X(4) X(8) X(9) X(13)

bool nphi_supported(int nphi) {
    switch (nphi) {
#define PF_CASE(n) case n:
        PF_NPHI_LIST(PF_CASE)
#undef PF_CASE
        return true;
    default: return false;
    }
}

int supported_nphi_list(int *out, int cap) {
    int n = 0;
#define PF_PUSH(v) { if (n < cap && out) out[n] = v; ++n; }
    PF_NPHI_LIST(PF_PUSH)
#undef PF_PUSH
    return n;
}

template <typename T>
hipError_t launch_stage(int dim, int nphi, const StageArgs<T> &args, int nblocks,
                        hipStream_t stream) {
    const dim3 grid(nblocks), block(256);
    switch (nphi) {
#define PF_CASE(n)                                                                    \
    case n:                                                                           \
        if (dim == 3)                                                                 \
            hipLaunchKernelGGL((stage_kernel<T, 3, n>), grid, block, 0, stream, args); \
        else                                                                          \
            hipLaunchKernelGGL((stage_kernel<T, 2, n>), grid, block, 0, stream, args); \
        break;
        PF_NPHI_LIST(PF_CASE)
#undef PF_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_embed_est(const DevParams<T> *P, int nphi, int with_c, long long V,
                            const T *unew, const T *z, const T *uold, T r_phi, T a_phi, T r_c,
                            T a_c, double *red, long long *redn, int nblocks,
                            hipStream_t stream) {
    hipLaunchKernelGGL(embed_kernel<T>, dim3(nblocks), dim3(256), 0, stream, P, nphi, with_c,
                       V, unew, z, uold, r_phi, a_phi, r_c, a_c, red, redn);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const T *u, int nphi, int with_c, long long V, double *red,
                       int nblocks, hipStream_t stream) {
    hipLaunchKernelGGL(diag_kernel<T>, dim3(nblocks), dim3(256), 0, stream, u, nphi, with_c,
                       V, red);
    return hipGetLastError();
}

hipError_t launch_finalize_norm(const double *red, const long long *redn, int nparts,
                                double *out, hipStream_t stream) {
    hipLaunchKernelGGL(finalize_norm_kernel, dim3(1), dim3(256), 0, stream, red, redn, nparts,
                       out);
    return hipGetLastError();
}

hipError_t launch_finalize_diag(const double *red, int nparts, double *out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(finalize_diag_kernel, dim3(1), dim3(256), 0, stream, red, nparts, out);
    return hipGetLastError();
}

template hipError_t launch_stage<float>(int, int, const StageArgs<float> &, int, hipStream_t);
template hipError_t launch_stage<double>(int, int, const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_embed_est<float>(const DevParams<float> *, int, int, long long,
                                            const float *, const float *, const float *, float,
                                            float, float, float, double *, long long *, int,
                                            hipStream_t);
template hipError_t launch_embed_est<double>(const DevParams<double> *, int, int, long long,
                                             const double *, const double *, const double *,
                                             double, double, double, double, double *,
                                             long long *, int, hipStream_t);
template hipError_t launch_diag<float>(const float *, int, int, long long, double *, int,
                                       hipStream_t);
template hipError_t launch_diag<double>(const double *, int, int, long long, double *, int,
                                        hipStream_t);

}  // namespace pf
