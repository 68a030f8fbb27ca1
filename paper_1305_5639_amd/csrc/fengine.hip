// F-engine: channelising FFT (Section 2, Eq. 1) with a fused requantise
// epilogue that writes the X-engine's time-blocked planar spectra layout.
//
// One workgroup of TH threads (256, or 512 for some int8 / FP8 sizes)
// transforms T = TH PT / C consecutive spectra of
// one input (64 KB of complex64 voltages, one contiguous coalesced run); every
// thread holds PT = 32 complex values.  The FFT is a Stockham autosort transform
// with radices up to 32 done in registers: one pass for C <= 32, two for
// C <= 1024 (one LDS round trip), three above.  The first pass reads straight
// from global memory; the others read and write LDS rows whose index is padded
// (one slot every 16 or 32, plus a few per row, chosen per C) so that the
// strided Stockham stores and loads are free of bank conflicts.  The last pass
// maps neighbouring lanes to neighbouring spectra of one channel; its values
// are scaled by inv_s[k], rounded to the spectra element type and staged in
// LDS as [plane][channel][spectrum], which turns the channel-major FFT output
// into runs of consecutive spectra per (channel, input, plane) row of the
// X-engine layout.  From kGatherMinC channels on, a workgroup's staged output
// goes instead to a scratch buffer in workgroup order, and fgather_kernel
// assembles the rows from those pieces.
//
// Twiddles between passes are float32 values of exp(-j 2 pi m / C) computed
// in float64 on the host: log2(R) table reads per butterfly, the other powers
// as products (at most log2(R) - 1 deep).  The twiddles inside a radix-R
// butterfly are constants.  Workgroups are numbered XCD-major (each XCD takes
// a contiguous range of work items), so the workgroups that fill the same
// 128-byte spectra rows run on one XCD at about the same time and their
// partial-row stores merge in that XCD's L2.
//
// Real-input form (Section 5: 8-bit real samples, transform length 2C): the
// 2C samples of a block are read as C complex values z[n] = x[2n] + j x[2n+1]
// straight from the int8 stream, transformed by the same C-point FFT, and the
// length-2C spectrum's channels k < C are split out of it after the last
// pass (one more LDS round trip for the partner value Z[C - k]).
#include "corr_internal.h"

#include <algorithm>

namespace corr {
namespace {

// The complex FP32 form at 2048 and 4096 channels stores straight into the
// held rows from 512-thread workgroups (8 or 4 spectra each, so 32- or
// 16-byte pieces of each row) instead of through the chunked gather: on 2^28
// samples 1.83 -> 1.64 ms at 2048 and 2.05 -> 1.93 ms at 4096 channels, and
// 30.7 -> 28.6 ms for 1024 inputs x 4096 channels x 1024 spectra.  At 8192
// channels (2 spectra per workgroup) the gather stays faster (2.36 against
// 2.94 ms), and so it does for every low-precision form, whose larger
// workgroups measured 35-75% slower.
template <int C, int PREC, bool REAL>
constexpr bool fp32_direct() {
    return !REAL && PREC == P_FP32 && (C == 2048 || C == 4096);
}

// Threads per workgroup: 256, or 512 for the int8 / FP8 complex forms at C =
// 512 and 1024, where twice the spectra per workgroup (so half as many
// partial output rows) measured 3-10% faster on 2^28 samples; at 256 channels
// they gained nothing; and 512 for fp32_direct.  From 2048 channels the
// chunked store and gather leave no partial rows to save.
template <int C, int PREC, bool REAL>
constexpr int threads() {
    if (fp32_direct<C, PREC, REAL>()) return 512;
    return (!REAL && (PREC == P_INT8 || PREC == P_FP8) && (C == 512 || C == 1024)) ? 512 : 256;
}

// Complex values per thread.  64 once paid at C >= 4096, where 32 left a
// workgroup so few spectra that its held-row stores went out in 1- to
// 4-byte pieces; with the chunked store and gather used from 2048 channels
// on, 32 (no spills) is faster at every size (4096 channels x 1024 inputs x
// 1024 FP8: 16.2 -> 14.5 ms; 8192 x 256 x 128 int8: 1.53 -> 1.15 ms).  A
// workgroup of TH threads transforms T = TH PT / C spectra; the helpers below
// recover PT as T C / TH.
template <int C, int PREC, bool REAL>
constexpr int per_thread() {
    return 32;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(-j 2 pi k / 32), k = 0..15.
__constant__ const float kW32[16][2] = {
    {1.000000000f, -0.000000000f},  {0.980785280f, -0.195090322f},  {0.923879533f, -0.382683432f},
    {0.831469612f, -0.555570233f},  {0.707106781f, -0.707106781f},  {0.555570233f, -0.831469612f},
    {0.382683432f, -0.923879533f},  {0.195090322f, -0.980785280f},  {0.000000000f, -1.000000000f},
    {-0.195090322f, -0.980785280f}, {-0.382683432f, -0.923879533f}, {-0.555570233f, -0.831469612f},
    {-0.707106781f, -0.707106781f}, {-0.831469612f, -0.555570233f}, {-0.923879533f, -0.382683432f},
    {-0.980785280f, -0.195090322f},
};

// x * exp(-j 2 pi k / R) for a compile-time k / R, with the trivial angles exact.
template <int R, int K>
__device__ __forceinline__ float2 rot(float2 x) {
    constexpr int k32 = K * (32 / R);                  // angle in units of 2 pi / 32, < 16
    if constexpr (k32 == 0) return x;
    else if constexpr (k32 == 8) return make_float2(x.y, -x.x);      // -j
    else return cmul(x, make_float2(kW32[k32][0], kW32[k32][1]));
}

// Forward R-point DFT in registers (R a power of two, <= 32), decimation in
// time: two R/2-point DFTs of the even and odd samples joined by W_R^k.
template <int R> struct Dft {
    template <int K = 0>
    static __device__ __forceinline__ void join(float2 *v, const float2 *e, const float2 *o) {
        if constexpr (K < R / 2) {
            const float2 t = rot<R, K>(o[K]);
            v[K] = cadd(e[K], t);
            v[K + R / 2] = csub(e[K], t);
            join<K + 1>(v, e, o);
        }
    }
    static __device__ __forceinline__ void run(float2 *v) {
        if constexpr (R == 1) {
            return;
        } else if constexpr (R == 2) {
            const float2 a = v[0], b = v[1];
            v[0] = cadd(a, b);
            v[1] = csub(a, b);
        } else {
            float2 e[R / 2], o[R / 2];
#pragma unroll
            for (int i = 0; i < R / 2; ++i) {
                e[i] = v[2 * i];
                o[i] = v[2 * i + 1];
            }
            Dft<R / 2>::run(e);
            Dft<R / 2>::run(o);
            join(v, e, o);
        }
    }
};

// Radices of the passes (product C, each <= 32) and the LDS row padding:
// element i of a row is stored at i + (i >> SH), rows are C + (C >> SH) + EX
// apart.  The paddings come from a bank-mapping simulation of every pass.
template <int C> struct Plan;
template <> struct Plan<16> { static constexpr int NP = 1, R0 = 16, R1 = 1, R2 = 1, SH = 5, EX = 0; };
template <> struct Plan<32> { static constexpr int NP = 1, R0 = 32, R1 = 1, R2 = 1, SH = 5, EX = 0; };
template <> struct Plan<64> { static constexpr int NP = 2, R0 = 8, R1 = 8, R2 = 1, SH = 5, EX = 1; };
template <> struct Plan<128> { static constexpr int NP = 2, R0 = 8, R1 = 16, R2 = 1, SH = 4, EX = 1; };
template <> struct Plan<256> { static constexpr int NP = 2, R0 = 16, R1 = 16, R2 = 1, SH = 4, EX = 1; };
template <> struct Plan<512> { static constexpr int NP = 2, R0 = 16, R1 = 32, R2 = 1, SH = 4, EX = 1; };
template <> struct Plan<1024> { static constexpr int NP = 2, R0 = 32, R1 = 32, R2 = 1, SH = 5, EX = 2; };
template <> struct Plan<2048> { static constexpr int NP = 3, R0 = 8, R1 = 16, R2 = 16, SH = 4, EX = 4; };
template <> struct Plan<4096> { static constexpr int NP = 3, R0 = 16, R1 = 16, R2 = 16, SH = 4, EX = 8; };
template <> struct Plan<8192> { static constexpr int NP = 3, R0 = 8, R1 = 32, R2 = 32, SH = 5, EX = 0; };

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Butterfly q of thread tid in a pass of radix R maps to (spectrum t, index
// j), with b = tid + TH q (TH threads per workgroup):
//   MAP_PLAIN : (b / (C/R), b % (C/R));
//   MAP_REMAP : (b % T, b / T), the last pass, so that neighbouring lanes hold
//               neighbouring spectra of one channel;
//   MAP_PAIRED: the last pass of the real-input form when C/R >= 2 and the Q
//               butterflies of a thread are even in number: t = tid % T, and
//               with g = tid / T, G = TH / T, butterfly q < Q/2 takes
//               j = g + G q while butterfly Q-1-q takes its mirror C/R - j (C/R/2
//               in place of the mirror of j = 0), so a thread holds channel k
//               and channel C - k of the same spectrum together.
enum { MAP_PLAIN = 0, MAP_REMAP = 1, MAP_PAIRED = 2 };

template <int C, int T, int TH, int R, int MAP>
__device__ __forceinline__ void bfly_index(int tid, int q, int &t, int &j) {
    const int b = tid + TH * q;
    if constexpr (MAP == MAP_REMAP) {
        t = b % T;
        j = b / T;
    } else if constexpr (MAP == MAP_PAIRED) {
        constexpr int Q = T * C / TH / R, CR = C / R, G = TH / T;
        static_assert(T <= TH && Q % 2 == 0 && CR == G * Q, "paired mapping needs T | TH and even Q");
        t = tid % T;
        const int g = tid / T;
        if (q < Q / 2) {
            j = g + G * q;
        } else {
            const int j1 = g + G * (Q - 1 - q);
            j = j1 ? CR - j1 : CR / 2;
        }
    } else {
        t = b / (C / R);
        j = b % (C / R);
    }
}

// LDS index of element i of spectrum t (rows padded as Plan<C> says).
template <int C>
__device__ __forceinline__ int lidx(int t, int i) {
    using P = Plan<C>;
    return t * (C + (C >> P::SH) + P::EX) + i + (i >> P::SH);
}

// First Stockham pass, radix R: butterfly (t, j) takes x[t][j + r C/R] straight
// from global memory (spectra past n_spectra read as zero) and does an R-point
// DFT; no twiddles precede the first pass.  The loads are unconditional (a
// padding spectrum reads spectrum 0, which always exists, and is then zeroed)
// so that all of a thread's loads are in flight together: a load under a
// branch whose value is converted inside it would be waited for one by one.
__device__ __forceinline__ float2 to_f2(float2 x) { return x; }
__device__ __forceinline__ float2 to_f2(char2 x) { return make_float2((float)x.x, (float)x.y); }

// Plain or non-temporal (streaming) load of one input element.
template <bool NT>
__device__ __forceinline__ float2 ld_in(const float2 *p) {
    if constexpr (NT) {
        const unsigned long long u = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
        float2 r;
        __builtin_memcpy(&r, &u, sizeof r);
        return r;
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ char2 ld_in(const char2 *p) {
    return *p;
}

template <int C, int T, int TH, int R, bool NT, typename Src>
__device__ __forceinline__ void first_pass(float2 *v, const Src *__restrict__ src, int a0, int n_spectra,
                                           int tid) {
    constexpr int Q = T * C / TH / R, CR = C / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int t, j;
        bfly_index<C, T, TH, R, MAP_PLAIN>(tid, q, t, j);
        float2 *x = v + q * R;
        const bool ok = (a0 + t) < n_spectra;
        const Src *row = src + (int64_t)(ok ? a0 + t : 0) * C + j;
        Src raw[R];
#pragma unroll
        for (int r = 0; r < R; ++r) raw[r] = ld_in<NT>(row + r * CR);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float2 f = to_f2(raw[r]);
            x[r] = make_float2(ok ? f.x : 0.f, ok ? f.y : 0.f);
        }
        Dft<R>::run(x);
    }
}

// A later pass of radix R after NS points have been combined: butterfly (t, j)
// (already holding x[t][j + r C/R]) multiplies element r by
// W_C^(r (j mod NS) C/(NS R)) and does an R-point DFT.
template <int C, int T, int TH, int R, int NS, int MAP>
__device__ __forceinline__ void later_pass(float2 *v, const float2 *__restrict__ tw, int tid) {
    constexpr int Q = T * C / TH / R;
    constexpr int LR = ilog2(R);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int t, j;
        bfly_index<C, T, TH, R, MAP>(tid, q, t, j);
        float2 *x = v + q * R;
        const int m = (j % NS) * (C / (NS * R));
        float2 wp[LR];                                 // W^(m 2^i)
#pragma unroll
        for (int i = 0; i < LR; ++i) wp[i] = tw[m << i];
        float2 w[R];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const int hb = 31 - __builtin_clz(r);
            w[r] = (r == (1 << hb)) ? wp[hb] : cmul(w[r - (1 << hb)], wp[hb]);
            x[r] = cmul(x[r], w[r]);
        }
        Dft<R>::run(x);
    }
}

// Stockham reordering between a pass (radix R1 after NS1 points) and the next
// (radix R2): butterfly (t, j) of the first writes element r to
// x[t][(j/NS1) NS1 R1 + j mod NS1 + r NS1], butterfly (t', j') of the next
// reads x[t'][j' + r C/R2].  SPLIT: the LDS holds one float per element, so
// the real parts go first and the imaginary parts second, each component read
// back taking the registers of one just written (half the LDS, so more
// workgroups per CU); otherwise whole complex values in one round.
// wait_first: the LDS may still be read by an earlier exchange.
template <int C, int T, int TH, int R1, int NS1, int R2, int MAP2, bool SPLIT>
__device__ __forceinline__ void exchange(float2 *v, float *lds, int tid, bool wait_first) {
    constexpr int PT = T * C / TH;
    constexpr int Q1 = PT / R1, Q2 = PT / R2, CR2 = C / R2;
    if constexpr (!SPLIT) {
        float2 *l2 = reinterpret_cast<float2 *>(lds);
        if (wait_first) __syncthreads();
#pragma unroll
        for (int q = 0; q < Q1; ++q) {
            int t, j;
            bfly_index<C, T, TH, R1, MAP_PLAIN>(tid, q, t, j);
            const int base = (j / NS1) * NS1 * R1 + (j % NS1);
#pragma unroll
            for (int r = 0; r < R1; ++r) l2[lidx<C>(t, base + r * NS1)] = v[q * R1 + r];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q2; ++q) {
            int t, j;
            bfly_index<C, T, TH, R2, MAP2>(tid, q, t, j);
#pragma unroll
            for (int r = 0; r < R2; ++r) v[q * R2 + r] = l2[lidx<C>(t, j + r * CR2)];
        }
        return;
    }
    float xr[PT];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        if (comp == 1 || wait_first) __syncthreads();
#pragma unroll
        for (int q = 0; q < Q1; ++q) {
            int t, j;
            bfly_index<C, T, TH, R1, MAP_PLAIN>(tid, q, t, j);
            const int base = (j / NS1) * NS1 * R1 + (j % NS1);
#pragma unroll
            for (int r = 0; r < R1; ++r) lds[lidx<C>(t, base + r * NS1)] = comp ? v[q * R1 + r].y : v[q * R1 + r].x;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q2; ++q) {
            int t, j;
            bfly_index<C, T, TH, R2, MAP2>(tid, q, t, j);
#pragma unroll
            for (int r = 0; r < R2; ++r) {
                const float e = lds[lidx<C>(t, j + r * CR2)];
                if (comp == 0) xr[q * R2 + r] = e;
                else v[q * R2 + r] = make_float2(xr[q * R2 + r], e);
            }
        }
    }
}

// Radix, butterflies per thread and index range of the last pass of Plan<C>,
// and how the real-input form finds the partner Z[C - k] of each Z[k]: in the
// same thread (MAP_PAIRED, or C/R = 1 where every butterfly has j = 0), else
// through LDS.
template <int C, int PT = 32> struct Last {
    using P = Plan<C>;
    static constexpr int RL = P::NP == 1 ? P::R0 : (P::NP == 2 ? P::R1 : P::R2);
    static constexpr int Q = PT / RL, CR = C / RL;
    static constexpr bool PAIRED = CR >= 2 && Q % 2 == 0;
    static constexpr bool REAL_VIA_LDS = CR >= 2 && Q % 2 == 1;
};

// The passes of Plan<C>; v ends with the last pass's outputs in registers,
// laid out by mapping LMAP.
template <int C, int T, int TH, bool SPLIT, int LMAP, bool NT, typename Src>
__device__ __forceinline__ void fft(float2 *v, float *lds, const Src *__restrict__ src, int a0, int n_spectra,
                                    const float2 *__restrict__ tw, int tid) {
    using P = Plan<C>;
    first_pass<C, T, TH, P::R0, NT>(v, src, a0, n_spectra, tid);
    if constexpr (P::NP == 2) {
        exchange<C, T, TH, P::R0, 1, P::R1, LMAP, SPLIT>(v, lds, tid, false);
        later_pass<C, T, TH, P::R1, P::R0, LMAP>(v, tw, tid);
    } else if constexpr (P::NP == 3) {
        exchange<C, T, TH, P::R0, 1, P::R1, MAP_PLAIN, SPLIT>(v, lds, tid, false);
        later_pass<C, T, TH, P::R1, P::R0, MAP_PLAIN>(v, tw, tid);
        exchange<C, T, TH, P::R1, P::R0, P::R2, LMAP, SPLIT>(v, lds, tid, true);
        later_pass<C, T, TH, P::R2, P::R0 * P::R1, LMAP>(v, tw, tid);
    }
}

// X[k] and X[C - k] of the length-2C real-input spectrum from z = Z[k],
// p = Z[C - k] of the C-point transform of z[n] = x[2n] + j x[2n+1] and
// w = W_2C^k = exp(-j pi k / C):
//   E = (z + conj p) / 2,  O = (z - conj p) / 2j,
//   X[k] = E + w O,  X[C - k] = conj(E - w O)   (W_2C^(C-k) = -conj w).
__device__ __forceinline__ void split_pair(float2 &z, float2 &p, float2 w) {
    const float er = 0.5f * (z.x + p.x), ei = 0.5f * (z.y - p.y);
    const float orr = 0.5f * (z.y + p.y), oi = 0.5f * (p.x - z.x);
    const float wr = w.x * orr - w.y * oi, wi = w.x * oi + w.y * orr;
    z = make_float2(er + wr, ei + wi);
    p = make_float2(er - wr, wi - ei);
}

// One last-pass butterfly with j = 0: u[r] = Z[r C/RL].  X[0] = Re Z[0] +
// Im Z[0] (real); X[C/2] = conj Z[C/2]; the others pair r with RL - r.
template <int C, int RL>
__device__ __forceinline__ void split_j0(float2 *u, const float2 *__restrict__ tw2) {
    constexpr int CR = C / RL;
    u[0] = make_float2(u[0].x + u[0].y, 0.f);
    if constexpr (RL >= 2) {
        u[RL / 2] = make_float2(u[RL / 2].x, -u[RL / 2].y);
#pragma unroll
        for (int r = 1; r < RL / 2; ++r) split_pair(u[r], u[RL - r], tw2[r * CR]);
    }
}

// Real-input split with every partner in the same thread (MAP_PAIRED, or
// C/R = 1).  In MAP_PAIRED butterfly q < Q/2 (index j) pairs element r with
// element RL-1-r of butterfly Q-1-q (index C/R - j); the thread with g = 0
// instead holds j = 0 in butterfly 0 and j = C/R/2 in butterfly Q-1, each
// paired with itself (r with RL - r, and r with RL-1-r).
template <int C, int T, int TH, int RL>
__device__ __forceinline__ void real_split_regs(float2 *v, const float2 *__restrict__ tw2, int tid) {
    constexpr int Q = T * C / TH / RL, CR = C / RL;
    if constexpr (CR == 1) {
#pragma unroll
        for (int q = 0; q < Q; ++q) split_j0<C, RL>(v + q * RL, tw2);
    } else {
        constexpr int G = TH / T;
        const int g = tid / T;
#pragma unroll
        for (int q = 0; q < Q / 2; ++q) {
            float2 *a = v + q * RL, *b = v + (Q - 1 - q) * RL;
            if (q == 0 && g == 0) {
                split_j0<C, RL>(a, tw2);
#pragma unroll
                for (int r = 0; r < RL / 2; ++r) split_pair(b[r], b[RL - 1 - r], tw2[CR / 2 + r * CR]);
            } else {
                const int j = g + G * q;
#pragma unroll
                for (int r = 0; r < RL; ++r) split_pair(a[r], b[RL - 1 - r], tw2[j + r * CR]);
            }
        }
    }
}

// Real-input split through LDS, for last passes whose butterflies per thread
// are odd in number (a single butterfly, so no pairing within the thread):
// with P = Z[(C - k) mod C] of the C-point transform Z of z[n] = x[2n] + j x[2n+1],
//   E = (Z[k] + conj P) / 2,  O = (Z[k] - conj P) / 2j,  X[k] = E + W_2C^k O,
// k < C, W_2C^k = exp(-j pi k / C) = tw2[k].  v holds Z[k] as the last pass
// left it (k = j + r C/RL of spectrum t, butterfly b = tid + TH q, (t, j) =
// (b % T, b / T)) and receives X[k] in the same places.  The partner values
// travel through LDS in natural [t][k] order, one component at a time when
// SPLIT.  The LDS may still be read by the last reordering on entry.
template <int C, int T, int TH, int RL, bool SPLIT>
__device__ __forceinline__ void real_split_lds(float2 *v, float *lds, const float2 *__restrict__ tw2, int tid) {
    constexpr int PT = T * C / TH;
    constexpr int Q = PT / RL, CR = C / RL;
    float pr[PT];                                      // partner real parts (SPLIT)
#pragma unroll
    for (int comp = 0; comp < (SPLIT ? 2 : 1); ++comp) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            int t, j;
            bfly_index<C, T, TH, RL, MAP_REMAP>(tid, q, t, j);
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int i = lidx<C>(t, j + r * CR);
                if constexpr (SPLIT) lds[i] = comp ? v[q * RL + r].y : v[q * RL + r].x;
                else reinterpret_cast<float2 *>(lds)[i] = v[q * RL + r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            int t, j;
            bfly_index<C, T, TH, RL, MAP_REMAP>(tid, q, t, j);
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int k = j + r * CR;
                const int i = lidx<C>(t, (C - k) & (C - 1));
                if (SPLIT && comp == 0) {
                    pr[q * RL + r] = lds[i];
                    continue;
                }
                float2 P;
                if constexpr (SPLIT) P = make_float2(pr[q * RL + r], lds[i]);
                else P = reinterpret_cast<const float2 *>(lds)[i];
                const float2 Z = v[q * RL + r];
                const float2 w = tw2[k];
                const float er = 0.5f * (Z.x + P.x), ei = 0.5f * (Z.y - P.y);
                const float orr = 0.5f * (Z.y + P.y), oi = 0.5f * (P.x - Z.x);
                v[q * RL + r] = make_float2(er + (w.x * orr - w.y * oi), ei + (w.x * oi + w.y * orr));
            }
        }
    }
}

// ---- requantisation --------------------------------------------------------
// OCP E4M3 (gfx950's FP8 format), round half to even, saturating at +-448: the
// value is clamped to the largest finite E4M3 magnitude first, so the
// hardware conversion (round to nearest even) never overflows.
__device__ __forceinline__ uint8_t to_e4m3(float y) {
    y = fminf(fmaxf(y, -448.0f), 448.0f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(y, y, 0, false) & 0xff);
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

// REAL: the input is int8 real samples (ld in bytes, block a at byte a*2C of
// its row) and tw2 holds exp(-j pi k / C); otherwise complex64 voltages (ld in
// complex samples, block a at sample a*C) and tw2 is unused.  inv_scale is
// never null (the host passes a table of ones for "no scale").
template <int C, int PREC, bool REAL>
__global__ __launch_bounds__((threads<C, PREC, REAL>())) __attribute__((amdgpu_waves_per_eu(
    PREC == P_FP32 || (REAL && Last<C>::REAL_VIA_LDS) || per_thread<C, PREC, REAL>() == 64 ? 2 : 3))) void fengine_kernel(
    const void *__restrict__ in, int64_t ld, int N, int n_spectra, int n_valid_pad,
    int n_work, const float *__restrict__ inv_scale,
    const float2 *__restrict__ tw, const float2 *__restrict__ tw2, uint8_t *__restrict__ spec, int64_t k_stride,
    int64_t t_stride, int tb0) {
    using E = typename Elem<PREC>::T;
    constexpr int TH = threads<C, PREC, REAL>();      // threads per workgroup
    constexpr int PT = per_thread<C, PREC, REAL>();   // complex values per thread
    constexpr int T = TH * PT / C;                     // spectra per workgroup
    using P = Plan<C>;
    static_assert(P::R0 * P::R1 * P::R2 == C, "radix plan must multiply to C");
    constexpr int RL = Last<C>::RL;                    // last radix
    constexpr int LMAP = REAL && Last<C>::PAIRED ? MAP_PAIRED : MAP_REMAP;
    constexpr int CP = C + (C >> P::SH) + P::EX;       // LDS row stride (floats)
    constexpr int ES = (int)sizeof(E);
    constexpr int TB = kRowBytes / ES;                 // spectra per time block
    constexpr int S = T * ES;                          // bytes of one staged row
    constexpr int CH = S < 16 ? S : 16;                // store chunk
    // The low-precision forms keep one float per element in LDS: the FFT's
    // reorderings move one component at a time, which halves the buffer so
    // three workgroups share a CU.  FP32, whose wider output staging needs the
    // registers that would allow that, keeps whole complex values (two
    // workgroups per CU, one round per reordering), and so does the
    // real-input form where the partners of its split step come through LDS.
    constexpr bool SPLIT = PREC != P_FP32 && !(REAL && Last<C>::REAL_VIA_LDS);
    // Two code-shape choices, both measured (MWA-like 256 x 1024 x 1000 and
    // 2048 streams x 256-point real transforms):
    //  - NT: the int8 / FP8 complex forms read the voltages with streaming
    //    (non-temporal) loads, 0.73 -> 0.64 ms; FP32 / FP16 and the
    //    real-input forms gain nothing or lose.
    //  - SCALE_TEST: the FP32 / FP16 complex forms keep a null test on the
    //    scale table (the host never passes null).  The compiler then loads
    //    the scales one pair at a time inside the staging loop, and the
    //    kernel's half-written spectra lines merge far better in L2: FP32
    //    writes 2.47 GB instead of 3.10 GB and takes 1.16 instead of
    //    1.53 ms (FP16 0.79 instead of 1.06 ms).  An explicit wait after each
    //    scale load recovers only part of that, and the other forms are
    //    faster without the test.
    constexpr bool NT = !REAL && (PREC == P_INT8 || PREC == P_FP8);
    constexpr bool SCALE_TEST = !REAL && (PREC == P_FP32 || PREC == P_FP16);
    // GATHER: stores go to the chunk scratch (passed as spec) in natural
    // order, [workgroup][plane][channel][spectrum], contiguous per workgroup.
    constexpr bool GATHER = C >= kGatherMinC && !fp32_direct<C, PREC, REAL>();
    static_assert(!GATHER || T <= TB, "a gathered workgroup must lie within one time block");
    constexpr int LF = SPLIT ? 1 : 2;                  // floats per LDS element
    constexpr int NPL = 2 * C * S <= T * CP * 4 * LF ? 2 : 1;   // planes staged at a time
    static_assert(NPL * C * S <= T * CP * 4 * LF, "staging must fit the FFT buffer");

    __shared__ __attribute__((aligned(16))) float lds[T * CP * LF];
    const int tid = threadIdx.x;

    // XCD-major work order: XCD x = blockIdx % 8 takes items [x*per, (x+1)*per).
    // Items run input-fastest within a time block, GPT workgroups per (time
    // block, input): the workgroups running together on an XCD then fill
    // whole 128-byte lines (k, tb, p) of consecutive inputs, which merge in
    // its L2 and leave it as contiguous runs.
    constexpr int GPT = TB > T ? TB / T : 1;
    const int per = (n_work + 7) / 8;
    const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= n_work) return;
    const int rest = w / GPT;
    const int p = rest % N;
    const int a0 = ((rest / N) * GPT + w % GPT) * T;

    float2 v[PT];
    if constexpr (REAL) {
        const char2 *src = reinterpret_cast<const char2 *>(static_cast<const int8_t *>(in) + (int64_t)p * ld);
        fft<C, T, TH, SPLIT, LMAP, false>(v, lds, src, a0, n_spectra, tw, tid);
        if constexpr (Last<C>::REAL_VIA_LDS) real_split_lds<C, T, TH, RL, SPLIT>(v, lds, tw2, tid);
        else real_split_regs<C, T, TH, RL>(v, tw2, tid);
    } else {
        fft<C, T, TH, SPLIT, LMAP, NT>(v, lds, static_cast<const float2 *>(in) + (int64_t)p * ld, a0, n_spectra, tw,
                                   tid);
    }

    // v[q RL + r] holds channel k = j + r C/RL of spectrum t for last-pass
    // butterfly q, (t, j) as mapping LMAP gives them.  NPL planes at a time
    // are requantised and staged in LDS as [plane][channel][spectrum], then
    // stored as runs of consecutive spectra of each (channel, plane) row:
    // the row (k, tb, p, plane) at spec + tb t_stride + k k_stride + p 128 +
    // plane 64, or, for GATHER, the workgroup's staged block as it stands.
    constexpr int CR = C / RL;
    using V = typename Bytes<CH>::T;
    constexpr int CPR = S / CH;                        // chunks per staged row
    constexpr int NCH = NPL * C * CPR;
    uint8_t *stage = reinterpret_cast<uint8_t *>(lds);
#pragma unroll
    for (int pl0 = 0; pl0 < 2; pl0 += NPL) {
        __syncthreads();                               // every thread is done reading lds
#pragma unroll
        for (int q = 0; q < PT / RL; ++q) {
            int t, j;
            bfly_index<C, T, TH, RL, LMAP>(tid, q, t, j);
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int k = j + r * CR;
                const float sc = SCALE_TEST ? (inv_scale ? inv_scale[k] : 1.0f) : inv_scale[k];
                const float2 y = v[q * RL + r];
#pragma unroll
                for (int pp = 0; pp < NPL; ++pp)
                    *reinterpret_cast<E *>(stage + (pp * C + k) * S + t * ES) =
                        Elem<PREC>::conv((pl0 + pp ? y.y : y.x) * sc);
            }
        }
        __syncthreads();
        for (int c = tid; c < NCH; c += TH) {
            const int row = c / CPR, x = c % CPR;
            const int pl = pl0 + row / C, k = row % C;
            const int a = a0 + x * (CH / ES);
            if (a >= n_valid_pad) continue;
            const int tb = tb0 + a / TB, within = a % TB;
            uint8_t *dst = GATHER ? spec + (int64_t)w * (2 * C * S) + (int64_t)pl0 * C * S + (int64_t)c * CH
                                  : spec + (int64_t)tb * t_stride + (int64_t)k * k_stride +
                                        (int64_t)p * (2 * kRowBytes) + pl * kRowBytes + within * ES;
            *reinterpret_cast<V *>(dst) = *reinterpret_cast<const V *>(stage + c * CH);
        }
    }
}

// Second step of a gathered F-engine chunk: the scratch holds, for chunk time
// block tbl, chunk input i and piece g < GPT = 64 / S, workgroup w = (tbl np
// + i) GPT + g's [plane][channel][S-byte piece] (piece g = spectra g T ..
// g T + T - 1 of the block).  Each thread assembles one 16-byte quarter of a
// 64-byte row (k, tb, p, plane) from 16 / S pieces; four neighbouring lanes
// write one whole row.
template <int S>
__global__ __launch_bounds__(256) void fgather_kernel(const uint8_t *__restrict__ scr, uint8_t *__restrict__ spec,
                                                      int log2c, int np, int ntb, int64_t ks, int64_t ts,
                                                      int tb_first, int p0) {
    static_assert(S == 1 || S == 2 || S == 4 || S == 8 || S == 16, "piece size");
    constexpr int GPT = kRowBytes / S, PV = 16 / S;
    const int C = 1 << log2c;
    const int64_t wg_bytes = (int64_t)2 * C * S;
    const int64_t total = (int64_t)ntb * np * 2 * C * 4;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int v = (int)(e & 3);
        const int64_t r = e >> 2;
        const int row = (int)(r & (2 * C - 1));        // plane * C + k
        const int64_t r2 = r >> (log2c + 1);
        const int i = (int)(r2 % np), tbl = (int)(r2 / np);
        const uint8_t *src = scr + ((int64_t)(tbl * np + i) * GPT + v * PV) * wg_bytes + (int64_t)row * S;
        uint4 out;
        if constexpr (S == 16) {
            out = *reinterpret_cast<const uint4 *>(src);
        } else {
            using W = typename Bytes<S>::T;
            W piece[PV];
#pragma unroll
            for (int u = 0; u < PV; ++u) piece[u] = *reinterpret_cast<const W *>(src + u * wg_bytes);
            __builtin_memcpy(&out, piece, 16);
        }
        uint8_t *dst = spec + (int64_t)(tb_first + tbl) * ts + (int64_t)(row & (C - 1)) * ks +
                       (int64_t)(p0 + i) * (2 * kRowBytes) + (row >> log2c) * kRowBytes + v * 16;
        *reinterpret_cast<uint4 *>(dst) = out;
    }
}

template <int PREC, int C, bool REAL>
hipError_t launch_c(int N, const void *in, int64_t ld, int n_spectra, const float *inv_scale,
                    const float2 *tw, const float2 *tw2, void *spec, SpecLayout lay, FScratch scr, int tb0,
                    hipStream_t stream) {
    constexpr int TH = threads<C, PREC, REAL>();
    constexpr int T = TH * per_thread<C, PREC, REAL>() / C;
    const int TB = time_block(PREC);
    const int n_tb = (n_spectra + TB - 1) / TB;
    auto run = [&](const void *src, int n_in, int ns, uint8_t *dst, int first_tb) -> hipError_t {
        const int n_valid_pad = (ns + TB - 1) / TB * TB;
        const int groups = (n_valid_pad + T - 1) / T;
        const int64_t n_work = (int64_t)n_in * groups;
        if (n_work <= 0 || n_work > (int64_t)1 << 30) return hipErrorInvalidValue;
        const int grid = (int)((n_work + 7) / 8) * 8;
        hipLaunchKernelGGL((fengine_kernel<C, PREC, REAL>), dim3(grid), dim3(TH), 0, stream, src, ld, n_in, ns,
                           n_valid_pad, (int)n_work, inv_scale, tw, tw2, dst, lay.ks, lay.ts, first_tb);
        return hipGetLastError();
    };
    if constexpr (C < kGatherMinC || fp32_direct<C, PREC, REAL>()) {
        return run(in, N, n_spectra, static_cast<uint8_t *>(spec), tb0);
    } else {
        // Chunks of whole time blocks of all inputs, or of one time block of
        // a range of inputs, each filling at most the scratch.
        constexpr int S = T * (int)sizeof(typename Elem<PREC>::T);
        const int64_t unit = (int64_t)C * 2 * kRowBytes;
        if (!scr.buf || scr.bytes < unit) return hipErrorInvalidValue;
        const int np = (int)std::min<int64_t>(N, scr.bytes / unit);
        const int ntb = np == N ? (int)std::min<int64_t>(n_tb, scr.bytes / (unit * N)) : 1;
        int log2c = 0;
        while ((1 << log2c) < C) ++log2c;
        uint8_t *sb = static_cast<uint8_t *>(scr.buf);
        for (int tbc = 0; tbc < n_tb; tbc += ntb) {
            const int s0 = tbc * TB;
            const int ns = std::min(ntb * TB, n_spectra - s0);
            const int ntb_c = (ns + TB - 1) / TB;
            for (int p0 = 0; p0 < N; p0 += np) {
                const int npc = std::min(np, N - p0);
                const void *src = REAL ? static_cast<const void *>(static_cast<const int8_t *>(in) + p0 * ld +
                                                                   (int64_t)s0 * 2 * C)
                                       : static_cast<const void *>(static_cast<const float2 *>(in) + p0 * ld +
                                                                   (int64_t)s0 * C);
                hipError_t e = run(src, npc, ns, sb, 0);
                if (e != hipSuccess) return e;
                const int64_t total = (int64_t)ntb_c * npc * 2 * C * 4;
                const int64_t blocks = std::min<int64_t>((total + 255) / 256, (int64_t)1 << 20);
                hipLaunchKernelGGL(fgather_kernel<S>, dim3((unsigned)blocks), dim3(256), 0, stream, sb,
                                   static_cast<uint8_t *>(spec), log2c, npc, ntb_c, lay.ks, lay.ts, tb0 + tbc, p0);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
        }
        return hipSuccess;
    }
}

template <int PREC, bool REAL>
hipError_t launch_p(int C, int N, const void *in, int64_t ld, int n_spectra, const float *inv_scale,
                    const float2 *tw, const float2 *tw2, void *spec, SpecLayout lay, FScratch scr, int tb0,
                    hipStream_t stream) {
#define CORR_FENGINE_CASE(c)                                                                            \
    case c: return launch_c<PREC, c, REAL>(N, in, ld, n_spectra, inv_scale, tw, tw2, spec, lay, scr, tb0, stream);
    switch (C) {
        CORR_FENGINE_CASE(16)
        CORR_FENGINE_CASE(32)
        CORR_FENGINE_CASE(64)
        CORR_FENGINE_CASE(128)
        CORR_FENGINE_CASE(256)
        CORR_FENGINE_CASE(512)
        CORR_FENGINE_CASE(1024)
        CORR_FENGINE_CASE(2048)
        CORR_FENGINE_CASE(4096)
        CORR_FENGINE_CASE(8192)
    default: return hipErrorInvalidValue;
    }
#undef CORR_FENGINE_CASE
}

template <bool REAL>
hipError_t launch_any(int prec, int C, int N, const void *in, int64_t ld, int n_spectra, const float *inv_scale,
                      const float2 *tw, const float2 *tw2, void *spec, SpecLayout lay, FScratch scr, int tb0,
                      hipStream_t stream) {
    switch (prec) {
    case P_FP32: return launch_p<P_FP32, REAL>(C, N, in, ld, n_spectra, inv_scale, tw, tw2, spec, lay, scr, tb0, stream);
    case P_FP16: return launch_p<P_FP16, REAL>(C, N, in, ld, n_spectra, inv_scale, tw, tw2, spec, lay, scr, tb0, stream);
    case P_FP8: return launch_p<P_FP8, REAL>(C, N, in, ld, n_spectra, inv_scale, tw, tw2, spec, lay, scr, tb0, stream);
    case P_INT8: return launch_p<P_INT8, REAL>(C, N, in, ld, n_spectra, inv_scale, tw, tw2, spec, lay, scr, tb0, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fengine(int prec, int C, int N, const float2 *volts, int64_t ld, int n_spectra,
                          const float *inv_scale, const float2 *twiddle, void *spec, SpecLayout lay, FScratch scr,
                          int first_tb, hipStream_t stream) {
    return launch_any<false>(prec, C, N, volts, ld, n_spectra, inv_scale, twiddle, nullptr, spec, lay, scr, first_tb,
                             stream);
}

hipError_t launch_fengine_real8(int prec, int C, int N, const int8_t *samples, int64_t ld, int n_spectra,
                                const float *inv_scale, const float2 *twiddle, const float2 *twiddle2n, void *spec,
                                SpecLayout lay, FScratch scr, int first_tb, hipStream_t stream) {
    return launch_any<true>(prec, C, N, samples, ld, n_spectra, inv_scale, twiddle, twiddle2n, spec, lay, scr,
                            first_tb, stream);
}

}  // namespace corr
