// Data-movement kernels around the two engines: caller spectra in and out of
// the time-blocked planar layout, dump layout/order conversion, the s_k^2
// table and a zero fill.  None of these is on the F -> X hot path; the
// spectra moves are LDS-tiled transposes, the rest coalesced element maps.
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int kThreads = 256;


// Caller spectra <-> held rows.  For channel k and time block tb, the TB
// public rows a = tb*TB + t hold the 2N columns (2p + plane) of that channel
// contiguously; the held layout wants each column's TB values contiguous (one
// 64-byte plane row).  That is a TB x 2N transpose per (k, tb).  One
// workgroup moves a tile of kCols columns: TB public segments of kCols * ES
// bytes <-> kCols held rows of 64 bytes, 16 KB either way, through LDS.  Both
// sides move 16-byte vectors; the LDS row of public row t stores its 16-byte
// chunks XOR-swizzled by the held vector t falls in, so the gathers of one
// wave (16 columns x 4 held vectors) hit distinct banks.
constexpr int kCols = 256;

template <typename T>
__device__ __forceinline__ int lds_elem(int t, int j) {
    constexpr int ES = (int)sizeof(T), VE = 16 / ES, W = kCols * ES;
    const int byte = j * ES, chunk = byte >> 4;
    const int tg = (t / VE) & 3;
    return t * W + ((chunk ^ (tg * ES)) << 4) + (byte & 15);
}

// Byte-wise max(b, -127) of four int8 values: a byte equal to 0x80 (-128)
// becomes 0x81 (-127), every other byte is unchanged.  x marks the -128 bytes
// as zero bytes; the zero-byte test below is exact (no borrow between bytes).
__device__ __forceinline__ uint32_t sat_int8x4(uint32_t v) {
    const uint32_t x = v ^ 0x80808080u;
    const uint32_t nz = ((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x;
    return v | ((~nz & 0x80808080u) >> 7);
}

// INGEST: public src -> held dst (the tail of the last block zero-filled);
// else held src -> public dst.  VEC: public rows 16-byte aligned (2N * ES a
// multiple of 16, base aligned), so public segments move as vectors.  SAT8
// (int8 ingest): -128 is read as -127, the symmetric range the X-engine's
// exact negation and the int32 overflow bound assume.
template <typename T, bool INGEST, bool VEC, bool SAT8 = false>
__global__ __launch_bounds__(kThreads) void relayout_kernel(const uint8_t *__restrict__ src,
                                                             uint8_t *__restrict__ dst, int C, int N,
                                                             int n_spectra, int n_tb, int n_cc, SpecLayout lay) {
    constexpr int ES = (int)sizeof(T), TB = kRowBytes / ES, VE = 16 / ES, W = kCols * ES;
    constexpr int PUB_VECS = TB * (W / 16);             // 1024 either side
    __shared__ __align__(16) uint8_t lds[TB * W];
    const int64_t g = blockIdx.x;
    const int cc = (int)(g % n_cc);
    const int tb = (int)((g / n_cc) % n_tb);
    const int k = (int)(g / ((int64_t)n_cc * n_tb));
    const int cols = 2 * N, c_base = cc * kCols;
    const int64_t pub_row = (int64_t)cols * ES;         // bytes per public (a, k) row
    uint8_t *held = (INGEST ? dst : const_cast<uint8_t *>(src)) + (int64_t)tb * lay.ts + (int64_t)k * lay.ks;

    auto pub_addr = [&](int t, int col) -> int64_t {
        return ((int64_t)(tb * TB + t) * C + k) * pub_row + (int64_t)col * ES;
    };
    if (INGEST) {
        for (int i = threadIdx.x; i < PUB_VECS; i += kThreads) {
            const int t = i / (W / 16), c = i % (W / 16);
            const int a = tb * TB + t, col0 = c_base + c * VE;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (a < n_spectra && col0 < cols) {
                if (VEC && col0 + VE <= cols) {
                    v = *reinterpret_cast<const uint4 *>(src + pub_addr(t, col0));
                } else {
                    T e[VE];
                    for (int u = 0; u < VE; ++u)
                        e[u] = col0 + u < cols ? *reinterpret_cast<const T *>(src + pub_addr(t, col0 + u)) : T(0);
                    __builtin_memcpy(&v, e, 16);
                }
            }
            if constexpr (SAT8) {
                v.x = sat_int8x4(v.x);
                v.y = sat_int8x4(v.y);
                v.z = sat_int8x4(v.z);
                v.w = sat_int8x4(v.w);
            }
            *reinterpret_cast<uint4 *>(lds + lds_elem<T>(t, c * VE)) = v;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kCols * 4; i += kThreads) {
            const int j = i >> 2, hv = i & 3, col = c_base + j;
            if (col >= cols) continue;
            T e[VE];
            for (int u = 0; u < VE; ++u) e[u] = *reinterpret_cast<const T *>(lds + lds_elem<T>(hv * VE + u, j));
            uint4 v;
            __builtin_memcpy(&v, e, 16);
            *reinterpret_cast<uint4 *>(held + (int64_t)col * kRowBytes + hv * 16) = v;
        }
    } else {
        for (int i = threadIdx.x; i < kCols * 4; i += kThreads) {
            const int j = i >> 2, hv = i & 3, col = c_base + j;
            if (col >= cols) continue;
            const uint4 v = *reinterpret_cast<const uint4 *>(held + (int64_t)col * kRowBytes + hv * 16);
            T e[VE];
            __builtin_memcpy(e, &v, 16);
            for (int u = 0; u < VE; ++u) *reinterpret_cast<T *>(lds + lds_elem<T>(hv * VE + u, j)) = e[u];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < PUB_VECS; i += kThreads) {
            const int t = i / (W / 16), c = i % (W / 16);
            const int a = tb * TB + t, col0 = c_base + c * VE;
            if (a >= n_spectra || col0 >= cols) continue;
            const uint4 v = *reinterpret_cast<const uint4 *>(lds + lds_elem<T>(t, c * VE));
            if (VEC && col0 + VE <= cols) {
                *reinterpret_cast<uint4 *>(dst + pub_addr(t, col0)) = v;
            } else {
                T e[VE];
                __builtin_memcpy(e, &v, 16);
                for (int u = 0; u < VE && col0 + u < cols; ++u)
                    *reinterpret_cast<T *>(dst + pub_addr(t, col0 + u)) = e[u];
            }
        }
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
                                    int layout, int order, int is_int, const int *__restrict__ zflag) {
    const bool zero = zflag && *zflag;
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
        int2 v = zero ? make_int2(0, 0) : acc[(int64_t)k * Bl + (int64_t)ii * (ii + 1) / 2 + jj];
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

__global__ void dump_copy_kernel(const uint4 *__restrict__ acc, uint4 *__restrict__ dst, int64_t n_vec,
                                 const int *__restrict__ zflag) {
    const bool zero = *zflag != 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_vec; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = zero ? make_uint4(0, 0, 0, 0) : acc[e];
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

// nk: channels moved (the grid); C stays the channel stride of the public
// layout, so a public pointer advanced by k0 channels moves channels
// [k0, k0 + nk) to held channels [0, nk).
template <typename T, bool INGEST, bool SAT8 = false>
hipError_t relayout_t(int C, int N, int n_spectra, SpecLayout lay, const void *src, void *dst, hipStream_t s,
                      int nk = -1) {
    constexpr int TB = kRowBytes / (int)sizeof(T);
    const int n_tb = (n_spectra + TB - 1) / TB;
    const int n_cc = (2 * N + kCols - 1) / kCols;
    const int64_t grid = (int64_t)(nk < 0 ? C : nk) * n_tb * n_cc;
    if (grid < 1) return hipSuccess;
    if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const void *pub = INGEST ? src : dst;
    const bool vec = (2 * N * (int)sizeof(T)) % 16 == 0 && reinterpret_cast<uintptr_t>(pub) % 16 == 0;
    const uint8_t *in = static_cast<const uint8_t *>(src);
    uint8_t *out = static_cast<uint8_t *>(dst);
    if (vec)
        hipLaunchKernelGGL((relayout_kernel<T, INGEST, true, SAT8>), dim3((unsigned)grid), dim3(kThreads), 0, s, in,
                           out, C, N, n_spectra, n_tb, n_cc, lay);
    else
        hipLaunchKernelGGL((relayout_kernel<T, INGEST, false, SAT8>), dim3((unsigned)grid), dim3(kThreads), 0, s, in,
                           out, C, N, n_spectra, n_tb, n_cc, lay);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ingest(int prec, int C, int N, int n_spectra, SpecLayout lay, const void *src, void *spec,
                         hipStream_t stream) {
    switch (elem_bytes(prec)) {
    case 4: return relayout_t<uint32_t, true>(C, N, n_spectra, lay, src, spec, stream);
    case 2: return relayout_t<uint16_t, true>(C, N, n_spectra, lay, src, spec, stream);
    default:
        if (prec == P_INT8) return relayout_t<uint8_t, true, true>(C, N, n_spectra, lay, src, spec, stream);
        return relayout_t<uint8_t, true>(C, N, n_spectra, lay, src, spec, stream);
    }
}

hipError_t launch_ingest_channels(int prec, int C, int k0, int nk, int N, int n_spectra, SpecLayout lay,
                                  const void *src, void *spec, hipStream_t stream) {
    if (k0 < 0 || nk < 1 || k0 + nk > C) return hipErrorInvalidValue;
    const uint8_t *s0 = static_cast<const uint8_t *>(src) + (int64_t)k0 * 2 * N * elem_bytes(prec);
    switch (elem_bytes(prec)) {
    case 4: return relayout_t<uint32_t, true>(C, N, n_spectra, lay, s0, spec, stream, nk);
    case 2: return relayout_t<uint16_t, true>(C, N, n_spectra, lay, s0, spec, stream, nk);
    default:
        if (prec == P_INT8) return relayout_t<uint8_t, true, true>(C, N, n_spectra, lay, s0, spec, stream, nk);
        return relayout_t<uint8_t, true>(C, N, n_spectra, lay, s0, spec, stream, nk);
    }
}

hipError_t launch_export(int prec, int C, int N, int n_spectra, SpecLayout lay, const void *spec, void *dst,
                         hipStream_t stream) {
    switch (elem_bytes(prec)) {
    case 4: return relayout_t<uint32_t, false>(C, N, n_spectra, lay, spec, dst, stream);
    case 2: return relayout_t<uint16_t, false>(C, N, n_spectra, lay, spec, dst, stream);
    default: return relayout_t<uint8_t, false>(C, N, n_spectra, lay, spec, dst, stream);
    }
}

hipError_t launch_dump_convert(int C, int N, int layout, int order, int is_int, const void *acc, void *dst,
                               hipStream_t stream, const int *zflag) {
    const int64_t Bt = layout == 2 ? (int64_t)N * N : (int64_t)N * (N + 1) / 2;
    hipLaunchKernelGGL(dump_convert_kernel, dim3(grid_for(Bt * C)), dim3(kThreads), 0, stream,
                       static_cast<const int2 *>(acc), static_cast<int2 *>(dst), C, N, layout, order, is_int, zflag);
    return hipGetLastError();
}

hipError_t launch_dump_copy(const void *acc, void *dst, int64_t n_words, const int *zflag, hipStream_t stream) {
    // accumulators are 8-byte pairs, C * B of them; copy as 16-byte vectors
    // and finish an odd pair with the zero flag as a 2-word tail
    const int64_t n_vec = n_words / 4;
    hipLaunchKernelGGL(dump_copy_kernel, dim3(grid_for(n_vec)), dim3(kThreads), 0, stream,
                       static_cast<const uint4 *>(acc), static_cast<uint4 *>(dst), n_vec, zflag);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && n_words % 4) {
        hipLaunchKernelGGL(dump_convert_kernel, dim3(1), dim3(kThreads), 0, stream,
                           static_cast<const int2 *>(acc) + 2 * n_vec, static_cast<int2 *>(dst) + 2 * n_vec,
                           1, 1, 0, 0, 0, zflag);
        e = hipGetLastError();
    }
    return e;
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
