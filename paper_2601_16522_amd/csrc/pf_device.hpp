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

// Field f of vector v at a 32-bit per-lane byte offset, through a buffer
// resource: the descriptor (first plane of the field's group, group span in
// bytes) and the plane offset inside the group are uniform (scalar registers);
// fields of one group share one descriptor.  An offset past the group reads 0
// and drops a store instead of touching other memory.  0x00020000 is the
// buffer descriptor's format word for the gfx9 family.
// CP: cache-policy bits of the access (0: default; 2: non-temporal, for
// streams that are touched once).
template <int CP = 0>
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff,
                                          float) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, CP));
}
template <int CP = 0>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff,
                                           double) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, CP);
    return __hiloint2double((int)v[1], (int)v[0]);
}
template <int CP = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff,
                                          float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, (int)off, (int)soff, CP);
}
template <int CP = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff,
                                          double x) {
    typedef unsigned u2 __attribute__((vector_size(8)));
    u2 v;
    v[0] = (unsigned)__double2loint(x);
    v[1] = (unsigned)__double2hiint(x);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, (int)soff, CP);
}

// Buffer resource of group g of vector v: GS planes from its base.
// GS * plane_bytes < 2^32 by construction (set_field_bases).
template <typename T, int GS, typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t group_rsrc(const S &A, int v, int g) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(A.gb[v][g]), 0,
                                             (int)((unsigned)GS * A.plane_bytes), 0x00020000);
}

// Field f of vector v at per-lane byte offset boff, with GS planes per buffer
// group: group f / GS and plane f mod GS are constants wherever f is.
template <typename T, int GS, int CP = 0, typename S>
__device__ __forceinline__ T ldv(const S &A, int v, int f, unsigned boff) {
    const int g = f / GS;
    return buf_load<CP>(group_rsrc<T, GS>(A, v, g), boff, (unsigned)(f - g * GS) * A.plane_bytes, T(0));
}
template <typename T, int GS, int CP = 0, typename S>
__device__ __forceinline__ void stv(const S &A, int v, int f, unsigned boff, T x) {
    const int g = f / GS;
    buf_store<CP>(group_rsrc<T, GS>(A, v, g), boff, (unsigned)(f - g * GS) * A.plane_bytes, x);
}

template <typename T, int N, int GS, typename S>
__device__ __forceinline__ void load_point32(const S &A, int v, unsigned boff, bool withc, T *x) {
#pragma unroll
    for (int f = 0; f < N; ++f) x[f] = ldv<T, GS>(A, v, f, boff);
    x[N] = withc ? ldv<T, GS>(A, v, N, boff) : T(0);
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
