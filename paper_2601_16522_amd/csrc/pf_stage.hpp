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
// The path is a memory-bound stencil (a few flops per byte), so it uses no
// matrix cores.  Decomposition: a block is 256 threads covering a tile of
// tx x ty cells of the x-y plane; a wavefront spans 64 consecutive x cells
// (tx = 64) or two half rows (tx = 32), so every load and store of a plane row
// is coalesced.  In 3D a block marches through zchunk planes in z and keeps the
// planes z-1, z, z+1 of its own cells in registers: each value is read from HBM
// once per march plus the two halo planes.  x and y neighbours come from the
// L1/L2 caches (rows of the same tile are loaded by the block's other
// wavefronts; halo rows by the neighbouring tile, which the XCD-aware tile
// order places on the same XCD).
//
// Floating-point order: every sum is accumulated in a fixed order (phases
// ascending; neighbours x-, x+, y-, y+, z-, z+) and the library is compiled
// without contraction, so the double-precision kernels reproduce a sequential
// left-to-right evaluation of the same formulas bit for bit.
#pragma once

#include "pf_device.hpp"

namespace pf {

template <typename T, int DIM, int N, int KIND>
__device__ __forceinline__ void stage_body(const StageArgs<T> &A) {
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
            // activity: phase a takes part at the cell when phi_a > 0 at the cell
            // or at one of its 2d neighbours (the n(phi, grad phi) filter and N_z
            // of eq. phieq)
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

            // variational derivative delta_a = sum_{b != a} (A_ab Lap phi_b +
            // B_ab phi_b) + psi_{type(a)}(mu)
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
            // dphi_a/dt = -(1/N_z) sum_{b active} L_ab (delta_a - delta_b)
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
            T *__restrict__ out = A.out;
            T yv[N + 1];
            if constexpr (KIND == K_RHS) {
#pragma unroll
                for (int f = 0; f < N; ++f) out[f * V + idx] = r[f];
                if (withc) out[N * V + idx] = r[N];
            } else if constexpr (KIND == K_EST) {
                // e = (12 (u^n - u^{n+1}) + 6 dt (R0 + rhs(u^{n+1}))) / 15; a phi entry
                // whose trial value u^n + dt/2 (R0 + rhs(u^{n+1})) leaves [0,1] has
                // zero error; weights r max(|u^n|,|u^{n+1}|) + a; DoF count with
                // the two-DoF rule for cells without nontrivial phi entries
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
                if constexpr (KIND == K_EULER || KIND == K_SSP104_S5 || KIND == K_RKL2_FIRST) {
#pragma unroll
                    for (int f = 0; f <= N; ++f) yv[f] = cur[f] + A.a * r[f];
                } else if constexpr (KIND == K_SSP2_FINAL) {
                    const T *__restrict__ u0 = A.u0;
#pragma unroll
                    for (int f = 0; f <= N; ++f) {
                        const T u = (f < N || withc) ? u0[f * V + idx] : T(0);
                        yv[f] = ((A.a * cur[f] + u) + A.b * r[f]) / A.c;
                    }
                } else if constexpr (KIND == K_SSP104_FINAL) {
                    const T *__restrict__ u0 = A.u0;
#pragma unroll
                    for (int f = 0; f <= N; ++f) {
                        const T u = (f < N || withc) ? u0[f * V + idx] : T(0);
                        yv[f] = (u + A.a * cur[f]) + A.b * r[f];
                    }
                } else if constexpr (KIND == K_RKL1) {
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

                if constexpr (KIND == K_RKL2_FIRST) {
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
                } else if constexpr (KIND == K_SSP104_S5) {
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
                    if constexpr (KIND == K_EULER) {
                        if (A.out2 != nullptr) {
                            T *__restrict__ o2 = A.out2;
#pragma unroll
                            for (int f = 0; f < N; ++f) o2[f * V + idx] = r[f];
                            if (withc) o2[N * V + idx] = r[N];
                        }
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

    if constexpr (KIND == K_EST) {
        block_sum(acc, cnt);
        if (threadIdx.x == 0 && tile_ok) {
            A.red[L] = acc;
            A.redn[L] = cnt;
        }
    }
}

// One named kernel per stage kind, so that profiles separate them.
#define PF_STAGE_KERNEL(name, kind)                                                  \
    template <typename T, int DIM, int N>                                           \
    __global__ void __launch_bounds__(256) name(const StageArgs<T> A) {             \
        stage_body<T, DIM, N, kind>(A);                                             \
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

template <typename T, int DIM, int N>
hipError_t launch_stage_dn(const StageArgs<T> &A, int nblocks, hipStream_t stream) {
    const dim3 grid(nblocks), block(256);
    switch (A.kind) {
    case K_RHS: hipLaunchKernelGGL((rhs_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_EULER: hipLaunchKernelGGL((euler_stage_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_SSP2_FINAL: hipLaunchKernelGGL((ssp2_final_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_SSP104_S5: hipLaunchKernelGGL((ssp104_s5_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_SSP104_FINAL: hipLaunchKernelGGL((ssp104_final_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_RKL1: hipLaunchKernelGGL((rkl1_stage_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_RKL2_FIRST: hipLaunchKernelGGL((rkl2_first_stage_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_RKL2: hipLaunchKernelGGL((rkl2_stage_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    case K_EST: hipLaunchKernelGGL((estimator_kernel<T, DIM, N>), grid, block, 0, stream, A); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_stage_n(int dim, const StageArgs<T> &A, int nblocks, hipStream_t stream) {
    return dim == 3 ? launch_stage_dn<T, 3, N>(A, nblocks, stream)
                    : launch_stage_dn<T, 2, N>(A, nblocks, stream);
}

}  // namespace pf
