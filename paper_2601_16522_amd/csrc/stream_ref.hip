// stream_ref.hip -- streaming-bandwidth reference for the stage kernels.
//
// The stage kernels are bound by HBM streaming; the chip's published 8 TB/s
// is not what a streaming kernel reaches.  This program measures what plain,
// fully coalesced streaming kernels reach on the device, with the access mix
// of the dominant stage (four vectors read, one written: the RKL2 inner
// stage) and a footprint chosen by the caller (the stage's own vector size),
// so that a stage kernel can be compared with the best a simple stream does
// for the same traffic.  Kernels:
//   4r1w     o = a/2 + b/4 + c/8 + d/16, 4 B per lane (the stage kernels' width)
//   4r1w_nt  the same with non-temporal loads and stores
//   copy     o = a, 16 B per lane
//   read     sum of a, 16 B per lane (result kept by a never-taken store)
//   4r1w_planes  (with F NX NY) the stage kernels' access pattern without
//            their arithmetic: each vector holds F planes of NX x NY x NZ
//            values (NZ = N / (F NX NY)); a block of 256 threads takes a
//            64 x 4 tile of the x-y plane and marches 16 planes in z, reading
//            the F values of its cell from four vectors and writing them to
//            the fifth -- 5 F concurrent plane streams, where 4r1w has 5
// Usage: stream_ref N [reps [F NX NY]]; N = floats per vector.  Prints one
// JSON line with GB/s per kernel (bytes moved / mean launch time over reps
// launches, timed with HIP events after two warm-up launches).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                                \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) {                                                              \
            fprintf(stderr, "stream_ref: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            exit(1);                                                                         \
        }                                                                                    \
    } while (0)

__global__ void __launch_bounds__(256)
    k_4r1w(const float *__restrict__ a, const float *__restrict__ b, const float *__restrict__ c,
           const float *__restrict__ d, float *__restrict__ o, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = 0.5f * a[i] + 0.25f * b[i] + 0.125f * c[i] + 0.0625f * d[i];
}

__global__ void __launch_bounds__(256)
    k_4r1w_nt(const float *__restrict__ a, const float *__restrict__ b, const float *__restrict__ c,
              const float *__restrict__ d, float *__restrict__ o, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float v = 0.5f * __builtin_nontemporal_load(a + i) +
                        0.25f * __builtin_nontemporal_load(b + i) +
                        0.125f * __builtin_nontemporal_load(c + i) +
                        0.0625f * __builtin_nontemporal_load(d + i);
        __builtin_nontemporal_store(v, o + i);
    }
}

__global__ void __launch_bounds__(256)
    k_copy(const float4 *__restrict__ a, float4 *__restrict__ o, long long n4) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) o[i] = a[i];
}

__global__ void __launch_bounds__(256)
    k_read(const float4 *__restrict__ a, float *__restrict__ o, long long n4) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.f;
    if (i < n4) {
        const float4 x = a[i];
        s = x.x + x.y + x.z + x.w;
    }
    if (s == 12345.678f) o[0] = s;  // the input is zero-filled: never taken
}

template <int F>
__global__ void __launch_bounds__(256)
    k_planes(const float *__restrict__ a, const float *__restrict__ b, const float *__restrict__ c,
             const float *__restrict__ d, float *__restrict__ o, int nx, int ny, int nz, int zc) {
    const int ntx = (nx + 63) / 64, nty = (ny + 3) / 4;
    const int L = blockIdx.x;
    const int tix = L % ntx, tiy = (L / ntx) % nty, tiz = L / (ntx * nty);
    const int x = tix * 64 + (int)threadIdx.x % 64, y = tiy * 4 + (int)threadIdx.x / 64;
    if (x >= nx || y >= ny) return;
    const long long V = (long long)nx * ny * nz;
    const int z1 = min(tiz * zc + zc, nz);
    for (int z = tiz * zc; z < z1; ++z) {
        const long long i = ((long long)z * ny + y) * nx + x;
        float va[F], vb[F], vc[F], vd[F];
#pragma unroll
        for (int f = 0; f < F; ++f) {
            va[f] = a[f * V + i];
            vb[f] = b[f * V + i];
            vc[f] = c[f * V + i];
            vd[f] = d[f * V + i];
        }
#pragma unroll
        for (int f = 0; f < F; ++f) o[f * V + i] = 0.5f * va[f] + 0.25f * vb[f] + 0.125f * vc[f] + 0.0625f * vd[f];
    }
}

template <int F>
void launch_planes(float *const *p, int nx, int ny, int nz) {
    const int zc = 16;
    const unsigned g = (unsigned)((nx + 63) / 64) * (unsigned)((ny + 3) / 4) * (unsigned)((nz + zc - 1) / zc);
    hipLaunchKernelGGL(k_planes<F>, dim3(g), dim3(256), 0, 0, p[0], p[1], p[2], p[3], p[4], nx, ny, nz, zc);
}

bool planes_dispatch(int F, float *const *p, int nx, int ny, int nz) {
    switch (F) {
#define PF_F(k) case k: launch_planes<k>(p, nx, ny, nz); return true;
        PF_F(2) PF_F(3) PF_F(4) PF_F(5) PF_F(6) PF_F(7) PF_F(8) PF_F(9) PF_F(10) PF_F(11) PF_F(12)
        PF_F(13) PF_F(14) PF_F(15) PF_F(16) PF_F(17)
#undef PF_F
    default: return false;
    }
}

int main(int argc, char **argv) {
    const long long n = argc > 1 ? atoll(argv[1]) : (1LL << 30);
    const int reps = argc > 2 ? atoi(argv[2]) : 10;
    if (n < 1024 || n > (1LL << 33) || reps < 1) {
        fprintf(stderr, "stream_ref: N must be in [1024, 2^33], reps >= 1\n");
        return 2;
    }
    const int F = argc > 5 ? atoi(argv[3]) : 0;
    const int nx = argc > 5 ? atoi(argv[4]) : 0, ny = argc > 5 ? atoi(argv[5]) : 0;
    const long long nzl = F > 0 && nx > 0 && ny > 0 ? n / ((long long)F * nx * ny) : 0;
    if (argc > 5 && (F < 2 || F > 17 || nx < 1 || ny < 1 || nzl < 1 || nzl > (1 << 30))) {
        fprintf(stderr, "stream_ref: F must be in [2, 17] and N >= F NX NY\n");
        return 2;
    }
    const int nz = (int)nzl;
    const long long n4 = n / 4;  // the 16 B kernels cover the first 4*(N/4) floats
    float *p[5];
    for (int k = 0; k < 5; ++k) {
        CK(hipMalloc(&p[k], n * sizeof(float)));
        CK(hipMemset(p[k], 0, n * sizeof(float)));
    }
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const int T = 256;
    const unsigned g1 = (unsigned)((n + T - 1) / T), g4 = (unsigned)((n4 + T - 1) / T);
    auto time_it = [&](auto launch) {
        for (int w = 0; w < 2; ++w) launch();
        CK(hipGetLastError());
        CK(hipDeviceSynchronize());
        CK(hipEventRecord(e0));
        for (int r = 0; r < reps; ++r) launch();
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, e0, e1));
        return ms / reps / 1e3;  // seconds per launch
    };
    const double B = (double)n * sizeof(float), B4 = (double)n4 * 16.0;
    const double t1 = time_it([&] {
        hipLaunchKernelGGL(k_4r1w, dim3(g1), dim3(T), 0, 0, p[0], p[1], p[2], p[3], p[4], n);
    });
    const double t2 = time_it([&] {
        hipLaunchKernelGGL(k_4r1w_nt, dim3(g1), dim3(T), 0, 0, p[0], p[1], p[2], p[3], p[4], n);
    });
    const double t3 = time_it([&] {
        hipLaunchKernelGGL(k_copy, dim3(g4), dim3(T), 0, 0, (const float4 *)p[0], (float4 *)p[4], n4);
    });
    const double t4 = time_it([&] {
        hipLaunchKernelGGL(k_read, dim3(g4), dim3(T), 0, 0, (const float4 *)p[0], p[4], n4);
    });
    double planes = 0.0;
    if (nz > 0) {
        const double t5 = time_it([&] { planes_dispatch(F, p, nx, ny, nz); });
        planes = 5.0 * F * (double)nx * ny * nz * sizeof(float) / t5 / 1e9;
    }
    printf("{\"floats_per_vector\": %lld, \"4r1w\": %.1f, \"4r1w_nt\": %.1f, \"copy\": %.1f, "
           "\"read\": %.1f",
           n, 5 * B / t1 / 1e9, 5 * B / t2 / 1e9, 2 * B4 / t3 / 1e9, B4 / t4 / 1e9);
    if (nz > 0) printf(", \"4r1w_planes\": %.1f, \"planes\": [%d, %d, %d, %d]", planes, F, nx, ny, nz);
    printf("}\n");
    for (int k = 0; k < 5; ++k) CK(hipFree(p[k]));
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    return 0;
}
