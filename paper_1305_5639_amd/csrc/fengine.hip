// F-engine: channelising FFT (Section 2, Eq. 1) with a fused requantise
// epilogue that writes the X-engine's time-blocked planar spectra layout.
//
// One workgroup of 256 threads transforms T = 8192 / C consecutive spectra of
// one input (64 KB of complex64 voltages, read as one contiguous coalesced
// run).  The FFT is a Stockham autosort transform: a first pass of radix 2, 4
// or 8 read straight from global memory into registers, then radix-8 passes
// through LDS; the last pass leaves channel k = j + r*C/8 of each spectrum in
// registers.  There the value is scaled by inv_s[k], rounded to the spectra
// element type, and staged in LDS as [plane][channel][spectrum], which turns
// the channel-major FFT output into runs of consecutive spectra per
// (channel, input, plane) row of the X-engine layout.
//
// Twiddles are float32 values of exp(-j 2 pi m / C) computed in float64 on the
// host.  Workgroups are mapped XCD-major (each XCD takes a contiguous range of
// work items), so the workgroups that fill the same 128-byte spectra rows run
// on one XCD at about the same time and their partial-row stores merge in
// that XCD's L2.
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int kThreads = 256;
constexpr int kTC = 8192;               // complex values per workgroup
constexpr int kPerThread = kTC / kThreads;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by -j
__device__ __forceinline__ float2 mul_mj(float2 a) { return make_float2(a.y, -a.x); }

template <int R> __device__ __forceinline__ void dft(float2 *v);

template <> __device__ __forceinline__ void dft<2>(float2 *v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

// Forward 4-point DFT, twiddle e^{-j pi/2} = -j.
template <> __device__ __forceinline__ void dft<4>(float2 *v) {
    float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    float2 s13 = cadd(v[1], v[3]), d13 = mul_mj(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

// Forward 8-point DFT as two 4-point DFTs of the even and odd samples joined
// with w8^k = e^{-j pi k / 4}.
template <> __device__ __forceinline__ void dft<8>(float2 *v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e);
    dft<4>(o);
    const float c = 0.70710678118654752440f;
    float2 o1 = make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
    float2 o2 = mul_mj(o[2]);
    float2 o3 = make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
// Radix of the first pass so that the remaining passes are all radix 8.
template <int C> constexpr int first_radix() {
    return (ilog2(C) % 3 == 0) ? 8 : (ilog2(C) % 3 == 1 ? 2 : 4);
}

// One Stockham pass of radix R after NS points have been combined:
// butterfly (t, j) reads x[t][j + r C/R], twiddles element r by
// W^(r (j mod NS) C/(NS R)), and writes x[t][(j/NS) NS R + j mod NS + r NS].
// Spectrum t occupies LDS row t with a padded stride CP.  Butterfly b of a
// thread maps to (t, j) = (b / (C/R), b % (C/R)), except in the last pass
// (REMAP), where (t, j) = (b % T, b / T) so that neighbouring lanes hold
// neighbouring spectra of one channel for the transposing epilogue.
template <int C, int T, int R, bool REMAP>
__device__ __forceinline__ void bfly_index(int b, int &t, int &j) {
    if constexpr (REMAP) {
        t = b % T;
        j = b / T;
    } else {
        t = b / (C / R);
        j = b % (C / R);
    }
}

template <int C, int T, int R, int NS, bool REMAP>
__device__ __forceinline__ void pass_compute(float2 *v, const float2 *__restrict__ tw, int tid) {
    constexpr int Q = kPerThread / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if constexpr (NS > 1) {
            int t, j;
            bfly_index<C, T, R, REMAP>(tid + kThreads * q, t, j);
            const int m = (j % NS) * (C / (NS * R));
            if constexpr (R == 8) {
                // three table reads, the other powers by products (depth <= 2)
                const float2 w1 = tw[m], w2 = tw[2 * m], w4 = tw[4 * m];
                const float2 w3 = cmul(w1, w2);
                v[q * R + 1] = cmul(v[q * R + 1], w1);
                v[q * R + 2] = cmul(v[q * R + 2], w2);
                v[q * R + 3] = cmul(v[q * R + 3], w3);
                v[q * R + 4] = cmul(v[q * R + 4], w4);
                v[q * R + 5] = cmul(v[q * R + 5], cmul(w1, w4));
                v[q * R + 6] = cmul(v[q * R + 6], cmul(w2, w4));
                v[q * R + 7] = cmul(v[q * R + 7], cmul(w3, w4));
            } else {
#pragma unroll
                for (int r = 1; r < R; ++r) v[q * R + r] = cmul(v[q * R + r], tw[r * m]);
            }
        }
        dft<R>(v + q * R);
    }
}

template <int C, int T, int CP, int R, bool REMAP>
__device__ __forceinline__ void pass_load_lds(float2 *v, const float2 *lds, int tid) {
    constexpr int Q = kPerThread / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int t, j;
        bfly_index<C, T, R, REMAP>(tid + kThreads * q, t, j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q * R + r] = lds[t * CP + j + r * (C / R)];
    }
}

template <int C, int T, int CP, int R, int NS>
__device__ __forceinline__ void pass_store_lds(const float2 *v, float2 *lds, int tid) {
    constexpr int Q = kPerThread / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int t, j;
        bfly_index<C, T, R, false>(tid + kThreads * q, t, j);
        const int base = t * CP + (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[base + r * NS] = v[q * R + r];
    }
}

// Passes after the first: NS points already combined, radix 8 from here on.
template <int C, int T, int CP, int NS>
__device__ __forceinline__ void later_passes(float2 *v, float2 *lds, const float2 *__restrict__ tw, int tid) {
    constexpr bool LAST = NS * 8 == C;
    __syncthreads();
    pass_load_lds<C, T, CP, 8, LAST>(v, lds, tid);
    pass_compute<C, T, 8, NS, LAST>(v, tw, tid);
    if constexpr (!LAST) {
        __syncthreads();
        pass_store_lds<C, T, CP, 8, NS>(v, lds, tid);
        later_passes<C, T, CP, NS * 8>(v, lds, tw, tid);
    }
}

// ---- requantisation --------------------------------------------------------
// OCP E4M3, round half to even, saturating at +-448.  a / 2^q is exact, so the
// only rounding is rintf (round half to even).
__device__ __forceinline__ uint8_t to_e4m3(float y) {
    y = fminf(fmaxf(y, -448.0f), 448.0f);
    const uint32_t u = __float_as_uint(y);
    const uint8_t sign = (uint8_t)((u >> 31) << 7);
    const float a = fabsf(y);
    int e = (int)((u >> 23) & 0xff) - 127;       // exponent of the leading bit (a normal float)
    if (e < -6) e = -6;                          // E4M3 subnormals share the quantum 2^-9
    const int q = e - 3;
    int m = (int)rintf(ldexpf(a, -q));            // 0..16
    if (m == 0) return sign;                      // +-0
    int E = q + 10;                               // field for m in [8, 16)
    if (m >= 16) { m = 8; E += 1; }               // rounded up into the next binade
    if (m < 8) return sign | (uint8_t)m;          // subnormal (only when q == -9)
    return sign | (uint8_t)(E << 3) | (uint8_t)(m - 8);
}

template <int PREC> struct Elem;
template <> struct Elem<P_FP32> {
    using T = float;
    static __device__ __forceinline__ T conv(float y) { return y; }
};
template <> struct Elem<P_FP16> {
    using T = _Float16;
    static __device__ __forceinline__ T conv(float y) {
        return (_Float16)fminf(fmaxf(y, -65504.0f), 65504.0f);   // RNE, saturating
    }
};
template <> struct Elem<P_FP8> {
    using T = uint8_t;
    static __device__ __forceinline__ T conv(float y) { return to_e4m3(y); }
};
template <> struct Elem<P_INT8> {
    using T = int8_t;
    static __device__ __forceinline__ T conv(float y) {
        return (int8_t)fminf(fmaxf(rintf(y), -127.0f), 127.0f);  // RNE, symmetric clamp
    }
};

template <int NB> struct Bytes;
template <> struct Bytes<1> { using T = uint8_t; };
template <> struct Bytes<2> { using T = uint16_t; };
template <> struct Bytes<4> { using T = uint32_t; };
template <> struct Bytes<8> { using T = uint2; };
template <> struct Bytes<16> { using T = uint4; };

template <int C, int PREC>
__global__ __launch_bounds__(kThreads) void fengine_kernel(
    const float2 *__restrict__ volts, int64_t ld, int N, int n_spectra, int n_valid_pad,
    int groups_per_input, int n_work, const float *__restrict__ inv_scale,
    const float2 *__restrict__ tw, uint8_t *__restrict__ spec, int n_tb_cap) {
    using E = typename Elem<PREC>::T;
    constexpr int T = kTC / C;                         // spectra per workgroup
    constexpr int PAD = T >= 64 ? 1 : 64 / T;          // LDS row padding (float2)
    constexpr int CP = C + PAD;                        // LDS row stride (float2)
    constexpr int ES = (int)sizeof(E);
    constexpr int TB = kRowBytes / ES;                 // spectra per time block
    constexpr int S = T * ES;                          // bytes of one staged row
    constexpr int CH = S < 16 ? S : 16;                // store chunk
    constexpr int R0 = first_radix<C>();
    static_assert(R0 < C, "at least two passes");
    static_assert(2 * C * S <= T * CP * 8, "staging must fit the FFT buffer");

    __shared__ __attribute__((aligned(16))) float2 lds[T * CP];
    const int tid = threadIdx.x;

    // XCD-major work order: XCD x = blockIdx % 8 takes items [x*per, (x+1)*per).
    const int per = (n_work + 7) / 8;
    const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= n_work) return;
    const int p = w / groups_per_input;
    const int a0 = (w % groups_per_input) * T;

    float2 v[kPerThread];
    {
        constexpr int Q = kPerThread / R0;
        constexpr int CR = C / R0;
        const float2 *src = volts + (int64_t)p * ld;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int b = tid + kThreads * q;
            const int t = b / CR, j = b % CR;
            const bool ok = (a0 + t) < n_spectra;
            const float2 *row = src + (int64_t)(a0 + t) * C + j;
#pragma unroll
            for (int r = 0; r < R0; ++r) v[q * R0 + r] = ok ? row[r * CR] : make_float2(0.f, 0.f);
        }
        pass_compute<C, T, R0, 1, false>(v, tw, tid);
        pass_store_lds<C, T, CP, R0, 1>(v, lds, tid);
        later_passes<C, T, CP, R0>(v, lds, tw, tid);
    }
    // v now holds, for last-pass butterfly b = tid + 256 q, channel
    // k = j + r C/8 of spectrum t, with t = b % T and j = b / T.
    constexpr int CR = C / 8;
    __syncthreads();                                   // every thread is done reading lds
    uint8_t *stage = reinterpret_cast<uint8_t *>(lds); // [plane][k][T] elements
#pragma unroll
    for (int q = 0; q < kPerThread / 8; ++q) {
        const int b = tid + kThreads * q;
        const int t = b % T, j = b / T;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int k = j + r * CR;
            const float s = inv_scale ? inv_scale[k] : 1.0f;
            const float2 y = v[q * 8 + r];
            *reinterpret_cast<E *>(stage + (0 * C + k) * S + t * ES) = Elem<PREC>::conv(y.x * s);
            *reinterpret_cast<E *>(stage + (1 * C + k) * S + t * ES) = Elem<PREC>::conv(y.y * s);
        }
    }
    __syncthreads();

    // Store staged rows: chunk c covers bytes [c*CH, (c+1)*CH) of the stage,
    // i.e. row = plane*C + k and spectra a0 + x*CH/ES ...
    // Destination: spec[k][tb][p][plane][TB].
    using V = typename Bytes<CH>::T;
    constexpr int CPR = S / CH;                        // chunks per staged row
    constexpr int NCH = 2 * C * CPR;
    const int64_t k_stride = channel_stride(n_tb_cap, N);
    for (int c = tid; c < NCH; c += kThreads) {
        const int row = c / CPR, x = c % CPR;
        const int pl = row / C, k = row % C;
        const int a = a0 + x * (CH / ES);
        if (a >= n_valid_pad) continue;
        const int tb = a / TB, within = a % TB;
        uint8_t *dst = spec + (int64_t)k * k_stride + ((int64_t)tb * N + p) * (2 * kRowBytes) +
                       pl * kRowBytes + within * ES;
        *reinterpret_cast<V *>(dst) = *reinterpret_cast<const V *>(stage + c * CH);
    }
}

template <int PREC, int C>
hipError_t launch_c(int N, const float2 *volts, int64_t ld, int n_spectra, const float *inv_scale,
                    const float2 *tw, void *spec, int n_tb_cap, hipStream_t stream) {
    constexpr int T = kTC / C;
    const int TB = time_block(PREC);
    const int n_tb = (n_spectra + TB - 1) / TB;
    const int n_valid_pad = n_tb * TB;
    const int groups = (n_valid_pad + T - 1) / T;
    const int64_t n_work = (int64_t)N * groups;
    if (n_work <= 0 || n_work > (int64_t)1 << 30) return hipErrorInvalidValue;
    const int grid = (int)((n_work + 7) / 8) * 8;
    hipLaunchKernelGGL((fengine_kernel<C, PREC>), dim3(grid), dim3(kThreads), 0, stream, volts, ld, N,
                       n_spectra, n_valid_pad, groups, (int)n_work, inv_scale, tw,
                       static_cast<uint8_t *>(spec), n_tb_cap);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_p(int C, int N, const float2 *volts, int64_t ld, int n_spectra, const float *inv_scale,
                    const float2 *tw, void *spec, int n_tb_cap, hipStream_t stream) {
    switch (C) {
    case 16: return launch_c<PREC, 16>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 32: return launch_c<PREC, 32>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 64: return launch_c<PREC, 64>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 128: return launch_c<PREC, 128>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 256: return launch_c<PREC, 256>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 512: return launch_c<PREC, 512>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 1024: return launch_c<PREC, 1024>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 2048: return launch_c<PREC, 2048>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 4096: return launch_c<PREC, 4096>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    case 8192: return launch_c<PREC, 8192>(N, volts, ld, n_spectra, inv_scale, tw, spec, n_tb_cap, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fengine(int prec, int C, int N, const float2 *volts, int64_t ld, int n_spectra,
                          const float *inv_scale, const float2 *twiddle, void *spec, int n_tb_cap,
                          hipStream_t stream) {
    switch (prec) {
    case P_FP32: return launch_p<P_FP32>(C, N, volts, ld, n_spectra, inv_scale, twiddle, spec, n_tb_cap, stream);
    case P_FP16: return launch_p<P_FP16>(C, N, volts, ld, n_spectra, inv_scale, twiddle, spec, n_tb_cap, stream);
    case P_FP8: return launch_p<P_FP8>(C, N, volts, ld, n_spectra, inv_scale, twiddle, spec, n_tb_cap, stream);
    case P_INT8: return launch_p<P_INT8>(C, N, volts, ld, n_spectra, inv_scale, twiddle, spec, n_tb_cap, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace corr
