// pf_device.hpp -- device helpers shared by the gfx950 kernels.
#pragma once

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
template <typename T, int N, typename C>
__device__ __forceinline__ void mu_mc(const C &P, const T *v, T &mu, T &mc) {
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

// A field plane at a 32-bit byte offset: the plane base comes from the kernel
// arguments (scalar registers), the per-lane offset is one 32-bit VGPR, so each
// access is a single global load/store with a scalar base.  The handle refuses
// grids whose plane exceeds 4 GiB.
template <typename T>
__device__ __forceinline__ T ldp(const T *base, unsigned boff) {
    return *(const T *)((const char *)base + boff);
}
template <typename T>
__device__ __forceinline__ void stp(T *base, unsigned boff, T v) {
    *(T *)((char *)base + boff) = v;
}

template <typename T, int N>
__device__ __forceinline__ void load_point32(const T *const *fb, unsigned boff, bool withc, T *v) {
#pragma unroll
    for (int f = 0; f < N; ++f) v[f] = ldp(fb[f], boff);
    v[N] = withc ? ldp(fb[N], boff) : T(0);
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

}  // namespace pf
