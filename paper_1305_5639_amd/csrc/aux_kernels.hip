// Data-movement kernels around the two engines: caller spectra in and out of
// the time-blocked planar layout, dump layout/order conversion, the s_k^2
// table and a zero fill.  None of these is on the F -> X hot path; they are
// plain coalesced-write element maps.
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int kThreads = 256;

template <typename T> __device__ __forceinline__ T zero_of() { return T(0); }

// One thread per internal element (k, tb, p, plane, t): coalesced writes.
template <typename T>
__global__ void ingest_kernel(const T *__restrict__ src, T *__restrict__ spec, int C, int N, int n_spectra,
                              int n_tb, SpecLayout lay) {
    constexpr int TB = kRowBytes / (int)sizeof(T);
    const int64_t k_stride = lay.ks / (int64_t)sizeof(T), t_stride = lay.ts / (int64_t)sizeof(T);
    const int64_t total = (int64_t)C * n_tb * N * 2 * TB;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e % TB);
        int64_t r = e / TB;
        const int pl = (int)(r % 2);
        r /= 2;
        const int p = (int)(r % N);
        r /= N;
        const int tb = (int)(r % n_tb);
        const int k = (int)(r / n_tb);
        const int a = tb * TB + t;
        const T v = a < n_spectra ? src[(((int64_t)a * C + k) * N + p) * 2 + pl] : zero_of<T>();
        spec[tb * t_stride + k * k_stride + ((int64_t)p * 2 + pl) * TB + t] = v;
    }
}

// One thread per public element (a, k, p, plane): coalesced writes.
template <typename T>
__global__ void export_kernel(const T *__restrict__ spec, T *__restrict__ dst, int C, int N, int n_spectra,
                              SpecLayout lay) {
    constexpr int TB = kRowBytes / (int)sizeof(T);
    const int64_t k_stride = lay.ks / (int64_t)sizeof(T), t_stride = lay.ts / (int64_t)sizeof(T);
    const int64_t total = (int64_t)n_spectra * C * N * 2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int pl = (int)(e % 2);
        int64_t r = e / 2;
        const int p = (int)(r % N);
        r /= N;
        const int k = (int)(r % C);
        const int a = (int)(r / C);
        const int tb = a / TB, t = a % TB;
        dst[e] = spec[tb * t_stride + k * k_stride + ((int64_t)p * 2 + pl) * TB + t];
    }
}

// Row i of the pair index for a flat index over the layout's pairs.
__device__ __forceinline__ void pair_of(int layout, int N, int64_t b, int &i, int &j) {
    if (layout == 2) {  // full
        i = (int)(b / N);
        j = (int)(b % N);
    } else if (layout == 0) {  // lower: b = i(i+1)/2 + j
        int r = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((int64_t)r * (r + 1) / 2 > b) --r;
        while ((int64_t)(r + 1) * (r + 2) / 2 <= b) ++r;
        i = r;
        j = (int)(b - (int64_t)r * (r + 1) / 2);
    } else {  // upper: b = i N - i(i-1)/2 + (j - i)
        // row starts s(i) = i N - i(i-1)/2; find the largest i with s(i) <= b
        const double Nd = N;
        int r = (int)(((2.0 * Nd + 1.0) - sqrt((2.0 * Nd + 1.0) * (2.0 * Nd + 1.0) - 8.0 * (double)b)) * 0.5);
        if (r < 0) r = 0;
        if (r > N - 1) r = N - 1;
        auto s = [&](int x) { return (int64_t)x * N - (int64_t)x * (x - 1) / 2; };
        while (r > 0 && s(r) > b) --r;
        while (r + 1 < N && s(r + 1) <= b) ++r;
        i = r;
        j = (int)(b - s(r)) + r;
    }
}

__global__ void dump_convert_kernel(const int2 *__restrict__ acc, int2 *__restrict__ dst, int C, int N,
                                    int layout, int order, int is_int) {
    const int64_t Bl = (int64_t)N * (N + 1) / 2;
    const int64_t Bt = layout == 2 ? (int64_t)N * N : Bl;
    const int64_t total = Bt * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t b;
        int k;
        if (order == 0) {
            k = (int)(e / Bt);
            b = e % Bt;
        } else {
            b = e / C;
            k = (int)(e % C);
        }
        int i, j;
        pair_of(layout, N, b, i, j);
        const bool mirrored = j > i;
        const int ii = mirrored ? j : i, jj = mirrored ? i : j;
        int2 v = acc[(int64_t)k * Bl + (int64_t)ii * (ii + 1) / 2 + jj];
        if (mirrored) {  // C_ij = conj(C_ji)
            if (is_int)
                v.y = -v.y;
            else
                v.y = __float_as_int(-__int_as_float(v.y));
        }
        dst[e] = v;
    }
}

__global__ void scale2_kernel(const float *__restrict__ inv, float *__restrict__ s2, int C) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < C) {
        if (inv) {
            const double x = (double)inv[k];
            s2[k] = (float)(1.0 / (x * x));
        } else {
            s2[k] = 1.0f;
        }
    }
}

__global__ void zero_kernel(uint32_t *__restrict__ p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

int grid_for(int64_t n) {
    int64_t g = (n + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

template <typename T>
hipError_t ingest_t(int C, int N, int n_spectra, SpecLayout lay, const void *src, void *spec, hipStream_t s) {
    constexpr int TB = kRowBytes / (int)sizeof(T);
    const int n_tb = (n_spectra + TB - 1) / TB;
    const int64_t total = (int64_t)C * n_tb * N * 2 * TB;
    hipLaunchKernelGGL(ingest_kernel<T>, dim3(grid_for(total)), dim3(kThreads), 0, s, static_cast<const T *>(src),
                       static_cast<T *>(spec), C, N, n_spectra, n_tb, lay);
    return hipGetLastError();
}

template <typename T>
hipError_t export_t(int C, int N, int n_spectra, SpecLayout lay, const void *spec, void *dst, hipStream_t s) {
    const int64_t total = (int64_t)n_spectra * C * N * 2;
    hipLaunchKernelGGL(export_kernel<T>, dim3(grid_for(total)), dim3(kThreads), 0, s,
                       static_cast<const T *>(spec), static_cast<T *>(dst), C, N, n_spectra, lay);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ingest(int prec, int C, int N, int n_spectra, SpecLayout lay, const void *src, void *spec,
                         hipStream_t stream) {
    switch (elem_bytes(prec)) {
    case 4: return ingest_t<uint32_t>(C, N, n_spectra, lay, src, spec, stream);
    case 2: return ingest_t<uint16_t>(C, N, n_spectra, lay, src, spec, stream);
    default: return ingest_t<uint8_t>(C, N, n_spectra, lay, src, spec, stream);
    }
}

hipError_t launch_export(int prec, int C, int N, int n_spectra, SpecLayout lay, const void *spec, void *dst,
                         hipStream_t stream) {
    switch (elem_bytes(prec)) {
    case 4: return export_t<uint32_t>(C, N, n_spectra, lay, spec, dst, stream);
    case 2: return export_t<uint16_t>(C, N, n_spectra, lay, spec, dst, stream);
    default: return export_t<uint8_t>(C, N, n_spectra, lay, spec, dst, stream);
    }
}

hipError_t launch_dump_convert(int C, int N, int layout, int order, int is_int, const void *acc, void *dst,
                               hipStream_t stream) {
    const int64_t Bt = layout == 2 ? (int64_t)N * N : (int64_t)N * (N + 1) / 2;
    hipLaunchKernelGGL(dump_convert_kernel, dim3(grid_for(Bt * C)), dim3(kThreads), 0, stream,
                       static_cast<const int2 *>(acc), static_cast<int2 *>(dst), C, N, layout, order, is_int);
    return hipGetLastError();
}

hipError_t launch_scale2(int C, const float *inv_scale, float *scale2, hipStream_t stream) {
    hipLaunchKernelGGL(scale2_kernel, dim3((C + kThreads - 1) / kThreads), dim3(kThreads), 0, stream, inv_scale,
                       scale2, C);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, int64_t n_words, hipStream_t stream) {
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n_words)), dim3(kThreads), 0, stream, static_cast<uint32_t *>(p),
                       n_words);
    return hipGetLastError();
}

}  // namespace corr
