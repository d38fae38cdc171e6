// pf_kernels.hip -- reduction and diagnostic kernels, and the dispatch of the
// fused stage kernels (pf_stage.hpp) over the compiled numbers of order
// parameters.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "pf_device.hpp"

namespace pf {

// Device scratch of the allocation-free error norm (pf_error_norm_device_noalloc):
// its per-tile partial sums live here instead of in memory the handle
// allocates.  Each GPU holds its own copy for the life of the process.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Device address of this GPU's scratch array.  The array's name is only a
// host-side stand-in for it, so host code uses the address looked up here,
// once per device with that device current, and cached.
hipError_t scratch_address(void **ptr) {
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void *addr[MAXDEV] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
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
diag_kernel(const T *__restrict__ u, const T *__restrict__ cpl, int nphi, int withc, long long V,
            double *red) {
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
            const double c = (double)cpl[i];
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
// The norm kernel writes (sum, count, norm) and then, after a system-scope
// fence, the sequence number seq into out[3]: out is coherent host memory that
// the host polls.
__global__ void __launch_bounds__(256)
finalize_norm_kernel(const double *red, const long long *redn, int n, double *out, double seq) {
    double acc = 0.0;
    long long cnt = 0;
    // unrolled so that the loads of several partials are in flight at once;
    // each thread still adds its partials in index order
#pragma unroll 16
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        acc += red[i];
        cnt += redn[i];
    }
    block_sum(acc, cnt);
    if (threadIdx.x == 0) {
        out[0] = acc;
        out[1] = (double)cnt;
        out[2] = cnt > 0 ? sqrt(acc / (double)cnt) : 0.0;
        __threadfence_system();
        *(volatile double *)(out + 3) = seq;
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

// Norms of a batched adaptive step, one block per instance: its per-tile
// partials red[tile0 .. tile0 + ntiles) summed exactly as finalize_norm_kernel
// sums a single instance's (thread-strided in index order, then block_sum), so
// an instance's norm equals the one its single-instance run computes.
__global__ void __launch_bounds__(256)
finalize_norm_batch_kernel(const double *red, const long long *redn, const int *ctl, double *out) {
    const int i = blockIdx.x;
    const int *c = ctl + 4 * i;  // tile0, ntiles, active, accept
    double acc = 0.0;
    long long cnt = 0;
    if (c[2]) {
        const double *r = red + c[0];
        const long long *rn = redn + c[0];
        const int n = c[1];
#pragma unroll 16
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            acc += r[k];
            cnt += rn[k];
        }
    }
    block_sum(acc, cnt);
    if (threadIdx.x == 0) {
        out[3 * i] = acc;
        out[3 * i + 1] = (double)cnt;
        out[3 * i + 2] = cnt > 0 ? sqrt(acc / (double)cnt) : 0.0;
    }
}

// src[0 .. count) to host-visible memory, then the sequence number after it
// once every value is visible to the host.
__global__ void __launch_bounds__(256)
publish_kernel(const double *src, int count, double *host_out, double seq) {
    for (int k = threadIdx.x; k < count; k += blockDim.x) host_out[k] = src[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence_system();
        *(volatile double *)(host_out + count) = seq;
    }
}

// The new state of each accepted instance (blockIdx.y), len[i] elements from
// off[i], grid-strided over blockIdx.x.
template <typename T>
__global__ void __launch_bounds__(256)
batch_accept_kernel(const T *src, T *dst, const long long *off, const long long *len, const int *ctl) {
    const int i = blockIdx.y;
    if (!ctl[4 * i + 3]) return;
    const long long o = off[i], n = len[i];
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        dst[o + k] = src[o + k];
}

// ------------------------------------------------------------------------
// Dispatch over the compiled (dim, N) instances
// ------------------------------------------------------------------------

// The build may compile a subset (a debug library): -D'PF_NPHI_LIST(X)=...'
// and -D'PF_NG_LIST(X)=...' then name the instances it links.
#ifndef PF_NPHI_LIST
#define PF_NPHI_LIST(X) X(2) X(3) X(4) X(8) X(9) X(13)
#endif
#ifndef PF_NG_LIST
#define PF_NG_LIST(X) X(1) X(2) X(4)
#endif

// defined in pf_stage_inst.hip, one object per (N, number of buffer groups)
#define PF_DECLG(n, g)                                                                       \
    extern template hipError_t launch_stage_n<float, n, g>(int, const StageArgs<float> &, int, \
                                                           hipStream_t);                      \
    extern template hipError_t launch_stage_n<double, n, g>(int, const StageArgs<double> &,    \
                                                            int, hipStream_t);
#define PF_DECL(n) PF_DECLG(n, 1) PF_DECLG(n, 2) PF_DECLG(n, 4)
template <typename T, int N, int NG>
hipError_t launch_stage_n(int dim, const StageArgs<T> &A, int nblocks, hipStream_t stream);
template <typename T, int N>
hipError_t launch_batch_euler_n(const BatchArgs<T> &B, int nblocks, hipStream_t stream);
PF_NPHI_LIST(PF_DECL)
#undef PF_DECL
#undef PF_DECLG
#define PF_DECLB(n)                                                                        \
    extern template hipError_t launch_batch_euler_n<float, n>(const BatchArgs<float> &, int, \
                                                              hipStream_t);                \
    extern template hipError_t launch_batch_euler_n<double, n>(const BatchArgs<double> &,   \
                                                               int, hipStream_t);
PF_NPHI_LIST(PF_DECLB)
#undef PF_DECLB

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

template <typename T, int N>
hipError_t launch_stage_g(int dim, const StageArgs<T> &args, int nblocks, hipStream_t stream) {
    switch (args.ng) {
#define PF_CASE(g) case g: return launch_stage_n<T, N, g>(dim, args, nblocks, stream);
        PF_NG_LIST(PF_CASE)
#undef PF_CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_stage(int dim, int nphi, const StageArgs<T> &args, int nblocks,
                        hipStream_t stream) {
    switch (nphi) {
#define PF_CASE(n) case n: return launch_stage_g<T, n>(dim, args, nblocks, stream);
        PF_NPHI_LIST(PF_CASE)
#undef PF_CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_batch_euler(int nphi, const BatchArgs<T> &args, int nblocks, hipStream_t stream) {
    switch (nphi) {
#define PF_CASE(n) case n: return launch_batch_euler_n<T, n>(args, nblocks, stream);
        PF_NPHI_LIST(PF_CASE)
#undef PF_CASE
    default: return hipErrorInvalidValue;
    }
}

// Advances the batch step counter by k after a run of k batched stages (one
// thread, an ordinary vector store).
__global__ void batch_tick_kernel(int *step_base, int k) {
    if (threadIdx.x == 0) step_base[0] = step_base[0] + k;
}

hipError_t launch_batch_tick(int *step_base, int k, hipStream_t stream) {
    hipLaunchKernelGGL(batch_tick_kernel, dim3(1), dim3(64), 0, stream, step_base, k);
    return hipGetLastError();
}

template hipError_t launch_batch_euler<float>(int, const BatchArgs<float> &, int, hipStream_t);
template hipError_t launch_batch_euler<double>(int, const BatchArgs<double> &, int, hipStream_t);

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
hipError_t launch_diag(const T *u, const T *cpl, int nphi, int with_c, long long V, double *red,
                       int nblocks, hipStream_t stream) {
    hipLaunchKernelGGL(diag_kernel<T>, dim3(nblocks), dim3(256), 0, stream, u, cpl, nphi, with_c,
                       V, red);
    return hipGetLastError();
}

// Sparse phase storage (Sec. 3.1 "Phase-field details"): conversion of whole
// state vectors between the dense layout (N phase planes, then c) and the
// sparse one (c in plane 0, up to n_p nonzero phase values in planes 1..n_p in
// ascending phase order, a word of nibble phase ids per cell at byte offset
// ids_off).  Packing applies the storage rule of the stage kernels: a cell
// with more than n_p nonzero phases keeps the n_p largest (equal values: the
// lower phase), divided by their sum; cut counts such cells.
template <typename T>
__global__ void __launch_bounds__(256)
pack_sparse_kernel(const T *__restrict__ dense, T *__restrict__ sp, int nphi, int withc, long long V,
                   int n_p, unsigned long long ids_off, unsigned long long *cut) {
    unsigned *ids = (unsigned *)((char *)sp + ids_off);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
        T p[NMAX];
        int cnt = 0;
        for (int a = 0; a < nphi; ++a) {
            p[a] = dense[a * V + i];
            cnt += p[a] != T(0) ? 1 : 0;
        }
        if (cnt > n_p) {
            unsigned keep = 0u;
            for (int k = 0; k < n_p; ++k) {
                int m = -1;
                for (int a = 0; a < nphi; ++a)
                    if (!((keep >> a) & 1u) && p[a] != T(0) && (m < 0 || p[a] > p[m])) m = a;
                keep |= 1u << m;
            }
            T sum = T(0);
            for (int a = 0; a < nphi; ++a) {
                if (!((keep >> a) & 1u)) p[a] = T(0);
                sum = sum + p[a];
            }
            if (sum > T(0)) {
                if constexpr (std::is_same<T, float>::value) {
                    const T inv = __builtin_amdgcn_rcpf(sum);
                    for (int a = 0; a < nphi; ++a) p[a] = p[a] * inv;
                } else {
                    for (int a = 0; a < nphi; ++a) p[a] = p[a] / sum;
                }
            }
            if (cut) atomicAdd(cut, 1ull);
        }
        unsigned w = 0xFFFFFFFFu;
        int k = 0;
        for (int a = 0; a < nphi; ++a)
            if (p[a] != T(0)) {
                sp[(k + 1) * V + i] = p[a];
                w = (w & ~(15u << (4 * k))) | ((unsigned)a << (4 * k));
                ++k;
            }
        for (; k < n_p; ++k) sp[(k + 1) * V + i] = T(0);
        sp[i] = withc ? dense[nphi * V + i] : T(0);
        ids[i] = w;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
unpack_sparse_kernel(const T *__restrict__ sp, T *__restrict__ dense, int nphi, int withc, long long V,
                     int n_p, unsigned long long ids_off) {
    const unsigned *ids = (const unsigned *)((const char *)sp + ids_off);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
        for (int a = 0; a < nphi; ++a) dense[a * V + i] = T(0);
        const unsigned w = ids[i];
        for (int k = 0; k < n_p; ++k) {
            const unsigned id = (w >> (4 * k)) & 15u;
            if (id < (unsigned)nphi) dense[id * V + i] = sp[(k + 1) * V + i];
        }
        if (withc) dense[nphi * V + i] = sp[i];
    }
}

template <typename T>
hipError_t launch_pack_sparse(const T *dense, T *sp, int nphi, int with_c, long long V, int n_p,
                              unsigned long long ids_off, unsigned long long *cut,
                              hipStream_t stream) {
    hipLaunchKernelGGL(pack_sparse_kernel<T>, dim3(2048), dim3(256), 0, stream, dense, sp, nphi,
                       with_c, V, n_p, ids_off, cut);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_unpack_sparse(const T *sp, T *dense, int nphi, int with_c, long long V, int n_p,
                                unsigned long long ids_off, hipStream_t stream) {
    hipLaunchKernelGGL(unpack_sparse_kernel<T>, dim3(2048), dim3(256), 0, stream, sp, dense, nphi,
                       with_c, V, n_p, ids_off);
    return hipGetLastError();
}

hipError_t launch_finalize_norm(const double *red, const long long *redn, int nparts,
                                double *out, double seq, hipStream_t stream) {
    hipLaunchKernelGGL(finalize_norm_kernel, dim3(1), dim3(256), 0, stream, red, redn, nparts,
                       out, seq);
    return hipGetLastError();
}

hipError_t launch_finalize_norm_batch(const double *red, const long long *redn, const int *ctl, int n,
                                      double *out, hipStream_t stream) {
    if (n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(finalize_norm_batch_kernel, dim3(n), dim3(256), 0, stream, red, redn, ctl, out);
    return hipGetLastError();
}

hipError_t launch_publish(const double *src, int count, double *host_out, double seq,
                          hipStream_t stream) {
    hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(256), 0, stream, src, count, host_out, seq);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_accept(const T *src, T *dst, const long long *off, const long long *len,
                               const int *ctl, int n, long long max_len, hipStream_t stream) {
    if (n < 1 || n > 65535 || max_len < 1) return hipErrorInvalidValue;
    const long long bx = std::min<long long>((max_len + 1023) / 1024, 4096);
    hipLaunchKernelGGL((batch_accept_kernel<T>), dim3((unsigned)bx, (unsigned)n), dim3(256), 0, stream,
                       src, dst, off, len, ctl);
    return hipGetLastError();
}
template hipError_t launch_batch_accept<float>(const float *, float *, const long long *,
                                               const long long *, const int *, int, long long,
                                               hipStream_t);
template hipError_t launch_batch_accept<double>(const double *, double *, const long long *,
                                                const long long *, const int *, int, long long,
                                                hipStream_t);

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
template hipError_t launch_diag<float>(const float *, const float *, int, int, long long, double *,
                                       int, hipStream_t);
template hipError_t launch_diag<double>(const double *, const double *, int, int, long long, double *,
                                        int, hipStream_t);
template hipError_t launch_pack_sparse<float>(const float *, float *, int, int, long long, int,
                                              unsigned long long, unsigned long long *, hipStream_t);
template hipError_t launch_pack_sparse<double>(const double *, double *, int, int, long long, int,
                                               unsigned long long, unsigned long long *, hipStream_t);
template hipError_t launch_unpack_sparse<float>(const float *, float *, int, int, long long, int,
                                                unsigned long long, hipStream_t);
template hipError_t launch_unpack_sparse<double>(const double *, double *, int, int, long long, int,
                                                 unsigned long long, hipStream_t);

}  // namespace pf
