// X-engine: the correlation of Section 2, Eq. 2, over the triangle of
// non-redundant input pairs (Section 4), as a batched Hermitian rank-A update
// on MFMA:  for each channel k,  C_k += X_k^H X_k,  X_k = [A spectra x N inputs].
//
// Complex arithmetic on real MFMA.  With x = xr + j xi,
//   Re C_ij = sum_a xr_i xr_j + xi_i xi_j
//   Im C_ij = sum_a xr_i xi_j - xi_i xr_j
// so each 32x32 output block takes four real MFMAs per K step:
//   re += Ar*Br, re += Ai*Bi, im += Ar*Bi, im += Ai*(-Br),
// where A holds rows i (the conjugated input) and B columns j.  The negated
// operand is formed in registers (sign flip for float forms, a byte-wise SWAR
// negate for int8, exact because the int8 range is symmetric).
//
// Tiling.  A workgroup owns a TILE x TILE block (rows I, columns J <= I) of
// one channel's triangle, TILE = 64 or 128.  Its waves form a 2 x (TILE / 32)
// grid: each wave owns TILE / 2 rows and one 32-column block, as 32x32 MFMA
// blocks with separate real and imaginary accumulators (TILE = 128: 8 waves of
// 64 x 32, 512 threads; TILE = 64: 4 waves of 32 x 32).  On diagonal blocks
// the waves whose columns lie wholly right of their rows idle, and a wave
// whose first 32 rows do skips that row block.  The K loop walks time blocks
// through a two-slot LDS ring filled by direct global-to-LDS copies
// (global_load_lds_dwordx4): each stage holds the TILE unpadded 128-byte rows
// (both planes) of each operand, with each row's 16-byte chunks XOR-swizzled
// so that 16 consecutive rows cover all 64 LDS banks.  Every lane reads 32
// bytes per (row block, plane) per stage, which is one K step for FP8
// (32x32x64), two for int8 (32x32x32) and FP16 (32x32x16), and eight for FP32
// (32x32x2).  Because the same K assignment is used for both operands, the
// spectrum-to-slot order inside a stage does not matter.
//
// Workgroups map XCD-major (each XCD takes a contiguous range of
// (channel, block) items) so one channel's blocks share an L2.
// The epilogue scales by s_k^2 (float forms) and adds into the persistent
// lower-triangle accumulators (or writes them on the first call of an
// integration); autos get an exactly zero imaginary part, as Eq. 2 gives.
#include <algorithm>
#include <type_traits>

#include "corr_internal.h"

namespace corr {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Device-memory pointers in the global address space.  Loads and stores
// through them compile to global_* instructions even where the pointer was
// itself read from memory (a descriptor); a generic pointer would give flat_*
// instructions, which also count against the LDS wait counter and so make
// every LDS wait drain the prefetch loads as well.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const uint8_t gu8;
typedef __attribute__((address_space(1))) const u32x4 gu4;
typedef __attribute__((address_space(1))) const float gf32;

// LDS ring.  A stage is one time block of the TILE rows of both operand
// slabs: 128-byte rows (both planes), two slots.  Rows have no padding; the
// 16-byte chunk c of row r sits in slot c ^ swz(r).  A 16-byte-per-lane LDS
// read is served 16 lanes (16 consecutive rows here) per cycle from 64 banks
// of 4 bytes; swz makes those 16 rows cover all 64 banks.  A lane's fragment
// of one (row, plane) and stage is kNT = 2 chunks (32 bytes).
constexpr int kRB = 2 * kRowBytes;                     // LDS row bytes
constexpr int kCPP = kRowBytes / 16;                   // 16-byte chunks per plane
constexpr int kNT = 2;                                 // chunks per lane fragment
__device__ __forceinline__ int swz(int r) { return (r >> 1) & 7; }
// LDS of a block: two ring slots of 2 TILE rows.
constexpr int ring_bytes(int tile) { return 2 * 2 * tile * kRB; }

// Per-precision fragment type and MFMA step for NT chunks per lane.  A
// fragment feeds NSUB MFMAs (sub-step e of the fragment).  The same chunk to
// K-slot assignment is used for both operands, so which spectra share an MFMA
// does not matter.
template <int PREC, int NT> struct XT;

template <int NT> struct XT<P_FP32, NT> {
    using Acc = f32x16;
    typedef float Frag __attribute__((ext_vector_type(4 * NT)));   // 4 NT spectra
    static constexpr int NSUB = 4 * NT;
    static __device__ __forceinline__ Frag load(const uint8_t *p, const int *o) {
        Frag f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const f32x4 v = *reinterpret_cast<const f32x4 *>(p + o[t]);
#pragma unroll
            for (int i = 0; i < 4; ++i) f[4 * t + i] = v[i];
        }
        return f;
    }
    static __device__ __forceinline__ Frag neg(Frag b) { return -b; }
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int e) {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], c, 0, 0, 0);
    }
};

// FP16 and int8 share the integer fragment: NT x 16 bytes, one MFMA per chunk.
template <int PREC, int NT> struct XTInt {
    typedef int Frag __attribute__((ext_vector_type(4 * NT)));
    static constexpr int NSUB = NT;
    static __device__ __forceinline__ Frag load(const uint8_t *p, const int *o) {
        Frag f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const i32x4 v = *reinterpret_cast<const i32x4 *>(p + o[t]);
#pragma unroll
            for (int i = 0; i < 4; ++i) f[4 * t + i] = v[i];
        }
        return f;
    }
    static __device__ __forceinline__ i32x4 part(const Frag &f, int e) {
        return i32x4{f[4 * e], f[4 * e + 1], f[4 * e + 2], f[4 * e + 3]};
    }
};

template <int NT> struct XT<P_FP16, NT> : XTInt<P_FP16, NT> {
    using Acc = f32x16;
    using Frag = typename XTInt<P_FP16, NT>::Frag;
    static __device__ __forceinline__ Frag neg(Frag b) { return b ^ (int)0x80008000u; }
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int e) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, XTInt<P_FP16, NT>::part(a, e)),
                                                   __builtin_bit_cast(f16x8, XTInt<P_FP16, NT>::part(b, e)), c, 0,
                                                   0, 0);
    }
};

template <int NT> struct XT<P_INT8, NT> : XTInt<P_INT8, NT> {
    using Acc = i32x16;
    using Frag = typename XTInt<P_INT8, NT>::Frag;
    // Byte-wise 0 - b without borrows between bytes (exact: the range is +-127).
    static __device__ __forceinline__ Frag neg(Frag b) {
        return (Frag)((0x80808080u - ((__typeof__(b))b & 0x7f7f7f7f)) ^ (~b & (int)0x80808080u));
    }
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int e) {
        c = __builtin_amdgcn_mfma_i32_32x32x32_i8(XTInt<P_INT8, NT>::part(a, e), XTInt<P_INT8, NT>::part(b, e), c,
                                                  0, 0, 0);
    }
};

template <int NT> struct XT<P_FP8, NT> {
    static_assert(NT == 2, "the FP8 MFMA takes 32 bytes per lane");
    using Acc = f32x16;
    using Frag = i32x8;
    static constexpr int NSUB = 1;
    static __device__ __forceinline__ Frag load(const uint8_t *p, const int *o) {
        const i32x4 a = *reinterpret_cast<const i32x4 *>(p + o[0]);
        const i32x4 b = *reinterpret_cast<const i32x4 *>(p + o[1]);
        return Frag{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    }
    static __device__ __forceinline__ Frag neg(Frag b) { return b ^ (int)0x80808080u; }
    // Format code 0 = FP8 E4M3 for both operands; E8M0 scale 127 = 2^0.
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int) {
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
    }
};

// Wave layout of a TILE x TILE block: 2 x WC waves, each owning QS = TILE / 2
// rows (FR blocks of 32) and one 32-column block.  TILE = 128: 8 waves of
// 64 x 32; TILE = 64: 4 waves of 32 x 32.  Narrow waves keep the complex
// accumulators of a wave at 32 FR registers each for Re and Im, so four waves
// share each SIMD: while some wait at a barrier or on LDS, others issue MFMAs.
template <int TILE> struct WaveGrid {
    static constexpr int WC = TILE / 32;               // waves across the columns
    static constexpr int NW = 2 * WC;                  // waves
    static constexpr int THREADS = 64 * NW;
    static constexpr int FR = TILE / 64;               // 32-row blocks per wave
    static constexpr int QS = TILE / 2;                // rows per wave
};

// One stage of a wave's FR blocks of 32x32.  pa / pb point at the lane's row
// (row block 0) and column in the stage; off[plane][t] are the lane's
// swizzled chunk offsets in a row.  Four real products per block (Re += Ar Br
// + Ai Bi, Im += Ar Bi + Ai (-Br)).  The column fragment is read once, each
// row block's fragments just before its MFMAs, and (except for FP8, whose
// MFMA takes both chunks) one 16-byte chunk at a time, which keeps the live
// fragment registers few enough for four waves per SIMD.  SKIP = 1: a
// diagonal wave whose first row block lies wholly above the diagonal leaves
// it out; SKIP = 2: a wave whose last row block lies wholly past the inputs
// leaves that out.
template <int PREC, int FR, int SKIP, typename Acc>
__device__ __forceinline__ void wave_stage(Acc (&re)[FR], Acc (&im)[FR], const uint8_t *pa, const uint8_t *pb,
                                           const int (&off)[2][kNT]) {
    constexpr int NC = PREC == P_FP8 ? 1 : kNT;        // chunk groups per stage
    constexpr int NTC = kNT / NC;                      // chunks per fragment
    using X = XT<PREC, NTC>;
    // The compiler's MFMA / LDS-read interleaving strategies, chosen per form
    // by measurement: FP16 at 1024 x 4096 x 1024 17.27 -> 16.54 ms and at 512 x
    // 2048 x 2048 4.24 -> 4.14 ms (strategy 0); int8 at 512 x 2048 x 2048
    // 2.44 -> 2.38 ms and FP32 133.5 -> 132.8 ms (strategy 1).  FP8, whose
    // fragments take both chunks at once, spills under either and keeps none.
    if constexpr (PREC == P_FP16) __builtin_amdgcn_iglp_opt(0);
    else if constexpr (PREC == P_FP32 || PREC == P_INT8) __builtin_amdgcn_iglp_opt(1);
#pragma unroll
    for (int t = 0; t < NC; ++t) {
        const typename X::Frag b0 = X::load(pb, off[0] + t * NTC);
        const typename X::Frag b1 = X::load(pb, off[1] + t * NTC);
        const typename X::Frag nb = X::neg(b0);
#pragma unroll
        for (int f = 0; f < FR; ++f) {
            if ((SKIP == 1 && f == 0) || (SKIP == 2 && f == FR - 1)) continue;
            const typename X::Frag a0 = X::load(pa + f * 32 * kRB, off[0] + t * NTC);
            const typename X::Frag a1 = X::load(pa + f * 32 * kRB, off[1] + t * NTC);
#pragma unroll
            for (int e = 0; e < X::NSUB; ++e) {
                X::mfma(re[f], a0, b0, e);             // + xr_i xr_j
                X::mfma(im[f], a0, b1, e);             // + xr_i xi_j
                X::mfma(re[f], a1, b1, e);             // + xi_i xi_j
                X::mfma(im[f], a1, nb, e);             // - xi_i xr_j
            }
        }
    }
}

// Asynchronous copy of 16 bytes per lane from global memory into LDS at
// lds + 16 * lane (the LDS address is taken from M0).  Issued as inline
// assembly so that the compiler, which cannot tell ring slots apart, does not
// wait for every copy in flight before each LDS read; completion is awaited
// explicitly with wait_vm.  The kernels here give the compiler no other use
// of M0.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(gu8 *src, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(lds)
                 : "memory", "m0");
}

#pragma clang diagnostic pop

// Wait until at most n vector-memory operations of this wave are in flight.
template <int n> __device__ __forceinline__ void wait_vm() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

// Where a block's results go.  Triangle (RECT = false): the lower-triangle
// product i(i+1)/2 + j of rows and columns below N with j <= i, B per
// channel.  Rectangle (RECT = true): rows [r0, r_end) x columns [c0, c_end),
// row-major, (i - r0) (c_end - c0) + (j - c0), B per channel; the two ranges
// do not overlap, so no pair is an auto.
struct OutMap {
    int r0, r_end, c0, c_end;
};

// The whole K loop and epilogue of one TILE x TILE block of channel k, rows
// I0.., columns J0.., by the waves of WaveGrid<TILE>.
// Time blocks stream through a two-slot LDS ring by direct global-to-LDS
// copies: the copy of time block t + 1 is issued when block t starts and
// lands while its MFMAs run.  The copies bypass registers, so the block
// keeps two workgroups per CU.  A diagonal block copies its one slab of rows
// once and reads both operands from it.  Rows past N copy row N - 1;
// they only feed outputs that are not written.  In the last time block,
// spectra past the valid count are zeroed in LDS once it lands.
template <int PREC, int TILE, bool RECT = false>
__device__ __forceinline__ void tile(uint8_t *smem, const uint8_t *__restrict__ base_k, int64_t t_stride, int N,
                                     int n_tb, int tv,
                                     int I0, int J0, int k, const float *__restrict__ scale2,
                                     void *__restrict__ acc_out, const void *acc_in, int64_t B, int first_call,
                                     int tid,
                                     OutMap om = OutMap{}) {
    constexpr int NT = kNT, RB = kRB, CPP = kCPP;
    using Acc = typename XT<PREC, NT>::Acc;
    constexpr int ES = PREC == P_FP32 ? 4 : (PREC == P_FP16 ? 2 : 1);
    constexpr int TB = kRowBytes / ES;
    using G = WaveGrid<TILE>;
    constexpr int QS = G::QS, FR = G::FR, WC = G::WC, NW = G::NW, THREADS = G::THREADS;
    constexpr int OPB = TILE * RB;                      // one operand slab of a stage
    constexpr int STG = 2 * OPB;                        // one stage
    constexpr int L = STG / (NW * 1024);                // 1 KB copies per wave per stage
    static_assert(2 * STG == ring_bytes(TILE) && L < 64 && L % 2 == 0, "ring geometry");
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = wave / WC, wj = wave % WC;
    const int m = lane & 31, h = lane >> 5;
    const bool diag = !RECT && I0 == J0;
    // on a diagonal block, a wave whose columns all lie right of its rows
    // idles; one whose first 32 rows do skips that row block.  A wave whose
    // rows or columns all lie past the inputs (past the rectangle) idles; one
    // whose last 32 rows do skips that row block.
    const int rlim = RECT ? om.r_end : N, clim = RECT ? om.c_end : N;
    const bool dwave = FR > 1 && diag && 32 * wj > wi * QS + 31;
    const bool lwave = FR > 1 && I0 + wi * QS + (FR - 1) * 32 >= rlim;
    const bool active = !(diag && 32 * wj > wi * QS + QS - 1) && I0 + wi * QS < rlim && J0 + wj * 32 < clim &&
                        !(dwave && lwave);
    const int S = n_tb;                                 // stages

    // Copy j of this wave covers stage bytes [g KB, (g + 1) KB), g = NW j + wave;
    // lane l writes bytes 16 l of it: slab o, row r, slot sl, which holds
    // chunk c = sl ^ swz(r), i.e. bytes [16 (c % CPP), +16) of plane c / CPP.
    int rowoff[L];
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const int bo = (NW * j + wave) * 1024 + 16 * lane;
        const int o = bo / OPB, r = (bo % OPB) / RB, c = ((bo % RB) / 16) ^ swz(r);
        const int pr = min((o ? J0 : I0) + r, N - 1);
        rowoff[j] = pr * RB + (c / CPP) * kRowBytes + (c % CPP) * 16;
    }
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)smem;
    gu8 *const gbase = (gu8 *)base_k;
    // A diagonal block's two slabs are the same rows: it copies slab 0 only
    // (copies j < L / 2 cover stage bytes [0, OPB)) and reads both operands
    // from it.
    auto issue = [&](int t) {
        gu8 *src = gbase + (int64_t)t * t_stride;
        const uint32_t dst = lds0 + (uint32_t)((t & 1) * STG);
#pragma unroll
        for (int j = 0; j < L; ++j)
            if (!diag || j < L / 2)
                dma16(src + rowoff[j], __builtin_amdgcn_readfirstlane(dst + (uint32_t)((NW * j + wave) * 1024)));
    };
    // Zero spectra >= tv of the landed last time block.
    auto fix_tail = [&](int t) {
        uint8_t *sm = smem + (t & 1) * STG;
        for (int q = tid; q < STG / 16; q += THREADS) {
            const int bo = q * 16, r = (bo % OPB) / RB, c = ((bo % RB) / 16) ^ swz(r);
            const int first = ((c % CPP) * 16) / ES;     // spectrum index of the chunk's first element
            if (first + 16 / ES <= tv) continue;
            uint32_t *wd = reinterpret_cast<uint32_t *>(sm + bo);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                uint32_t msk = 0;
#pragma unroll
                for (int bb = 0; bb < 4; ++bb)
                    if (first + (4 * d + bb) / ES < tv) msk |= 0xffu << (8 * bb);
                wd[d] &= msk;
            }
        }
    };

    // The lane's fragment chunk offsets within a row (the rows of a fragment
    // read are m modulo 32, and swz depends on r mod 16 only).
    int off[2][NT];
#pragma unroll
    for (int pl = 0; pl < 2; ++pl)
#pragma unroll
        for (int t = 0; t < NT; ++t) off[pl][t] = 16 * ((pl * CPP + h * NT + t) ^ swz(m));

    Acc re[FR], im[FR];
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            re[f][r] = 0;
            im[f][r] = 0;
        }

    const uint8_t *pa0 = smem + (wi * QS + m) * RB;
    const uint8_t *pb0 = smem + (diag ? 0 : OPB) + (wj * 32 + m) * RB;
    const bool tail = tv < TB;

    __builtin_amdgcn_s_setprio(2);                     // (see the copies in the loop)
    issue(0);
    __builtin_amdgcn_s_setprio(0);
    for (int t = 0; t < S; ++t) {
        wait_vm<0>();                                   // this wave's copies of block t landed
        __syncthreads();                                // block t landed; the other slot is free
        // The copies go out at a raised wave priority, ahead of the MFMAs of
        // the other waves on the SIMD (FP32, 1024 x 4096 x 1024: 137.0 ->
        // 133.3 ms; the FP16, FP8 and int8 forms unchanged within 1%; the
        // first block's copies too: a further 0.2-1%).
        __builtin_amdgcn_s_setprio(2);
        if (t + 1 < S) issue(t + 1);
        __builtin_amdgcn_s_setprio(0);
        if (tail && t == S - 1) {
            fix_tail(t);
            __syncthreads();
        }
        if (active) {
            const int so = (t & 1) * STG;
            // one uniform branch per stage keeps the MFMA stream branch-free
            if (dwave)
                wave_stage<PREC, FR, 1>(re, im, pa0 + so, pb0 + so, off);
            else if (PREC != P_FP8 && lwave)           // (a third FP8 body would spill)
                wave_stage<PREC, FR, 2>(re, im, pa0 + so, pb0 + so, off);
            else
                wave_stage<PREC, FR, 0>(re, im, pa0 + so, pb0 + so, off);
        }
    }
    if (!active) return;

    // Epilogue: element r of a 32x32 block is (row 8(r/4) + 4h + r%4, column m).
    // Rows go in batches of EH; each batch's accumulator reads are issued
    // before any of its writes.  The writes are streaming (non-temporal) so
    // that they displace fewer of the spectra rows other blocks still read
    // from L2 (FP8, 1024 inputs x 4096 channels: 9.45 -> 9.1-9.3 ms).  Elements outside the triangle (rectangle) or
    // past N read a valid address and are not written.  Offsets within a
    // channel fit 32 bits (N(N+1)/2 and N^2 < 2^31 for N <= 8192).
    using E = typename std::conditional<PREC == P_INT8, int, float>::type;
    typedef E T2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) T2 gT2;
    gT2 *out = (gT2 *)acc_out + (int64_t)k * B;
    const gT2 *in = (const gT2 *)acc_in + (int64_t)k * B;   // the sums so far (== out except when dumping)
    const float s2 = (PREC != P_INT8 && scale2) ? ((gf32 *)scale2)[k] : 1.0f;
    const int j = J0 + wj * 32 + m;
    // rows of a block per batch of accumulator reads: all 16 where a wave has
    // one row block, 8 where it has two (the registers allow no more)
    constexpr int EH = FR == 1 ? 16 : 8;
#pragma unroll
    for (int f = 0; f < FR; ++f) {
        if ((dwave && f == 0) || (lwave && f == FR - 1)) continue;
#pragma unroll
        for (int hh = 0; hh < 16 / EH; ++hh) {
            int idx[EH];
            uint32_t ok = 0;
#pragma unroll
            for (int q = 0; q < EH; ++q) {
                const int r = EH * hh + q;
                const int i = I0 + wi * QS + f * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                bool inside;
                int o;
                if constexpr (RECT) {
                    inside = i < om.r_end && j < om.c_end;
                    o = (i - om.r0) * (om.c_end - om.c0) + (j - om.c0);
                } else {
                    inside = i < N && j <= i;
                    o = i * (i + 1) / 2 + j;
                }
                ok |= (uint32_t)inside << q;
                idx[q] = inside ? o : 0;
            }
            T2 old[EH];
            if (!first_call) {
#pragma unroll
                for (int q = 0; q < EH; ++q) old[q] = in[idx[q]];
            }
#pragma unroll
            for (int q = 0; q < EH; ++q) {
                const int r = EH * hh + q;
                const int i = I0 + wi * QS + f * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                T2 v;
                const bool auto_ = !RECT && i == j;
                if constexpr (PREC == P_INT8) {
                    v = T2{re[f][r], auto_ ? 0 : im[f][r]};
                } else {
                    v = T2{re[f][r] * s2, auto_ ? 0.0f : im[f][r] * s2};
                }
                if (!first_call) {
                    v.x += old[q].x;
                    v.y += old[q].y;
                }
                if ((ok >> q) & 1u) __builtin_nontemporal_store(v, &out[idx[q]]);
            }
        }
    }
}

// Lower-triangle block t of a tiling with blocks (bi, bj), bj <= bi, in the
// order (0,0), (1,0), (1,1), (2,0), ...
__device__ __forceinline__ void tri_block(int t, int &bi, int &bj) {
    int b = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (b * (b + 1) / 2 > t) --b;
    while ((b + 1) * (b + 2) / 2 <= t) ++b;
    bi = b;
    bj = t - b * (b + 1) / 2;
}

// zflag (may be null): a device flag that, when set, makes this the first
// call of an integration whatever first_call says (the accumulators of a
// batch sub-array are then logically zero, whatever they hold).
template <int PREC, int TILE>
__global__ __launch_bounds__(WaveGrid<TILE>::THREADS) __attribute__((amdgpu_waves_per_eu(4))) void xengine_kernel(
    const uint8_t *__restrict__ spec, int N, int n_tiles, int n_work, int n_tb, int tv,
    int64_t k_stride, int64_t t_stride, const float *__restrict__ scale2, void *__restrict__ acc_out,
    const void *acc_in, int64_t B, int first_call, const int *__restrict__ zflag) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[ring_bytes(TILE)];
    const int per = (n_work + 7) / 8;
    const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= n_work) return;
    const int k = w / n_tiles;
    int bi, bj;
    tri_block(w % n_tiles, bi, bj);
    const int fc = zflag && *zflag ? 1 : first_call;
    tile<PREC, TILE>(smem, spec + (int64_t)k * k_stride, t_stride, N, n_tb, tv, bi * TILE, bj * TILE, k, scale2,
                     acc_out, acc_in, B, fc, threadIdx.x);
}

// Rectangle X-engine: rows [r0, r0 + ni) against columns [c0, c0 + nj) in
// TILE x TILE blocks (nbi x nbj per channel), XCD-major like xengine_kernel.
template <int PREC, int TILE>
__global__ __launch_bounds__(WaveGrid<TILE>::THREADS) __attribute__((amdgpu_waves_per_eu(4))) void xengine_rect_kernel(
    const uint8_t *__restrict__ spec, int N, int nbi, int nbj, int n_work, int n_tb, int tv, int64_t k_stride,
    int64_t t_stride, const float *__restrict__ scale2, void *__restrict__ out, int64_t B, int first_call, OutMap om) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[ring_bytes(TILE)];
    const int per = (n_work + 7) / 8;
    const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= n_work) return;
    const int nb = nbi * nbj;
    const int k = w / nb, bi = (w % nb) / nbj, bj = w % nbj;
    tile<PREC, TILE, true>(smem, spec + (int64_t)k * k_stride, t_stride, N, n_tb, tv, om.r0 + bi * TILE,
                           om.c0 + bj * TILE, k,
                           scale2, out, out, B, first_call, threadIdx.x, om);
}

// Persistent X-engine over many sub-arrays with blocks of TILE inputs, so
// uneven sub-arrays share one launch.  Work items are (sub-array, channel,
// block); XCD x's queue holds channels [x C/8, (x+1) C/8) of every sub-array,
// so the blocks of one channel run on one XCD and share its L2.  A workgroup
// takes items from its own XCD's queue through that queue's atomic counter
// (the ticket for the next item is taken while the current one runs), and
// once it is drained from the other queues in turn; every workgroup ends
// after one failed take on each of the eight queues.  Within a queue the
// descriptors follow their sorted order (largest item first) and a workgroup
// finds its descriptor by binary search over the queue offsets.
template <int PREC, int TILE>
__global__ __launch_bounds__(WaveGrid<TILE>::THREADS) __attribute__((amdgpu_waves_per_eu(4))) void xengine_batched_kernel(
    const XQueue *__restrict__ plan, const XDesc *__restrict__ all_desc, unsigned int *__restrict__ counter) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[ring_bytes(TILE)];
    __shared__ unsigned int s_item;
    const int tid = threadIdx.x;
    const int n_desc = plan->n_desc;
    const XDesc *__restrict__ desc = all_desc + plan->desc_offset;
    const int home = blockIdx.x % kXcds;
    for (int s = 0; s < kXcds; ++s) {
        const int x = (home + s) % kXcds;
        unsigned int *cnt = counter + x * kCounterStride;
        const int64_t qlen = plan->qlen[x];
        if (tid == 0) s_item = atomicAdd(cnt, 1u);
        __syncthreads();
        // uniform across the workgroup: keep it (and the descriptor fields it
        // selects) in scalar registers
        int64_t item = (unsigned int)__builtin_amdgcn_readfirstlane((int)s_item);
        __syncthreads();                                // s_item free for reuse
        // the descriptor of the last item and its item range in this queue:
        // a workgroup's items rise, so most items reuse it without a search
        int cur = 0, cur_fc = 0;
        int64_t c_lo = 1, c_hi = 0;
        while (item < qlen) {
            // take the next ticket now; its latency overlaps this item's loads
            unsigned int next = 0;
            if (tid == 0) next = atomicAdd(cnt, 1u);
            if (item < c_lo || item >= c_hi) {
                int lo = 0, hi = n_desc - 1;            // last descriptor with qbegin[x] <= item
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (desc[mid].qbegin[x] <= item) lo = mid; else hi = mid - 1;
                }
                cur = lo;
                c_lo = desc[lo].qbegin[x];
                c_hi = lo + 1 < n_desc ? desc[lo + 1].qbegin[x] : qlen;
                // the sub-array's flag is cleared only after the launch, so
                // every item of it reads the same value
                const int *zf = desc[lo].zflag;
                cur_fc = zf && *(const __attribute__((address_space(1))) int *)zf ? 1 : desc[lo].first_call;
            }
            const XDesc &d = desc[cur];
            const int64_t local = item - d.qbegin[x];
            const int k = x * d.C / kXcds + (int)(local / d.n_tiles);
            int bi, bj;
            tri_block((int)(local % d.n_tiles), bi, bj);
            // an opaque copy of the thread index keeps the block body's
            // per-lane address arithmetic inside the loop instead of live
            // across it (which cost registers and occupancy)
            int t = tid;
            asm volatile("" : "+v"(t));
            tile<PREC, TILE>(smem, d.spec + (int64_t)k * d.k_stride, d.tb_stride, d.N, d.n_tb, d.tv, bi * TILE,
                             bj * TILE, k,
                             d.scale2, d.acc, d.acc, d.B, cur_fc, t);
            if (tid == 0) s_item = next;
            __syncthreads();                            // also: every wave is done with smem
            item = (unsigned int)__builtin_amdgcn_readfirstlane((int)s_item);
            __syncthreads();
        }
    }
}

__global__ void reset_counters_kernel(unsigned int *counter) { counter[threadIdx.x * kCounterStride] = 0u; }

// After a batched launch: clear the zero flag of every sub-array in the plan.
__global__ void clear_flags_kernel(const XQueue *__restrict__ plan, const XDesc *__restrict__ desc) {
    const int n = plan[0].n_desc + plan[1].n_desc;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (desc[i].zflag) *desc[i].zflag = 0;
}

__global__ void set_flag_kernel(int *flag, int v) { *flag = v; }

template <int PREC, int TILE>
hipError_t launch_x(int C, int N, int n_spectra, const void *spec, SpecLayout lay,
                    const float *scale2, void *acc, const void *acc_in, int first_call, const int *zflag,
                    hipStream_t stream) {
    const int TB = time_block(PREC);
    const int n_tb = (n_spectra + TB - 1) / TB;
    const int tv = n_spectra - (n_tb - 1) * TB;
    const int n_blk = (N + TILE - 1) / TILE;
    const int n_tiles = n_blk * (n_blk + 1) / 2;
    const int64_t n_work = (int64_t)C * n_tiles;
    if (n_tb <= 0 || n_work <= 0 || n_work > ((int64_t)1 << 30)) return hipErrorInvalidValue;
    const int grid = (int)((n_work + 7) / 8) * 8;
    const int64_t B = (int64_t)N * (N + 1) / 2;
    hipLaunchKernelGGL((xengine_kernel<PREC, TILE>), dim3(grid), dim3(WaveGrid<TILE>::THREADS), 0, stream,
                       static_cast<const uint8_t *>(spec), N, n_tiles, (int)n_work, n_tb, tv, lay.ks, lay.ts,
                       scale2, acc, acc_in, B, first_call, zflag);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_xp(int tile, int C, int N, int n_spectra, const void *spec, SpecLayout lay,
                     const float *scale2, void *acc, const void *acc_in, int first_call, const int *zflag,
                     hipStream_t stream) {
    if (tile == 64)
        return launch_x<PREC, 64>(C, N, n_spectra, spec, lay, scale2, acc, acc_in, first_call, zflag, stream);
    if (tile == 128)
        return launch_x<PREC, 128>(C, N, n_spectra, spec, lay, scale2, acc, acc_in, first_call, zflag, stream);
    return hipErrorInvalidValue;
}

}  // namespace

template <int PREC, int TILE>
hipError_t launch_rect_t(int C, int N, int n_spectra, const void *spec, SpecLayout lay, const float *scale2,
                         void *out, int first_call, int r0, int ni, int c0, int nj, hipStream_t stream) {
    const int TB = time_block(PREC);
    const int n_tb = (n_spectra + TB - 1) / TB;
    const int tv = n_spectra - (n_tb - 1) * TB;
    const int nbi = (ni + TILE - 1) / TILE, nbj = (nj + TILE - 1) / TILE;
    const int64_t n_work = (int64_t)C * nbi * nbj;
    if (n_tb <= 0 || n_work <= 0 || n_work > ((int64_t)1 << 30) || r0 < 0 || c0 < 0 || r0 + ni > N || c0 + nj > N)
        return hipErrorInvalidValue;
    const int grid = (int)((n_work + 7) / 8) * 8;
    hipLaunchKernelGGL((xengine_rect_kernel<PREC, TILE>), dim3(grid), dim3(WaveGrid<TILE>::THREADS), 0, stream,
                       static_cast<const uint8_t *>(spec), N, nbi, nbj, (int)n_work, n_tb, tv,
                       lay.ks, lay.ts, scale2, out, (int64_t)ni * nj, first_call,
                       OutMap{r0, r0 + ni, c0, c0 + nj});
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_rect_p(int tile, int C, int N, int n_spectra, const void *spec, SpecLayout lay,
                         const float *scale2, void *out, int first_call, int r0, int ni, int c0, int nj,
                         hipStream_t stream) {
    if (tile == 64)
        return launch_rect_t<PREC, 64>(C, N, n_spectra, spec, lay, scale2, out, first_call, r0, ni, c0, nj, stream);
    if (tile == 128)
        return launch_rect_t<PREC, 128>(C, N, n_spectra, spec, lay, scale2, out, first_call, r0, ni, c0, nj, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_xengine_rect(int prec, int tile, int C, int N, int n_spectra, const void *spec, SpecLayout lay,
                               const float *scale2, void *out, int first_call, int r0, int ni, int c0, int nj,
                               hipStream_t stream) {
    switch (prec) {
    case P_FP32: return launch_rect_p<P_FP32>(tile, C, N, n_spectra, spec, lay, scale2, out, first_call, r0, ni, c0, nj, stream);
    case P_FP16: return launch_rect_p<P_FP16>(tile, C, N, n_spectra, spec, lay, scale2, out, first_call, r0, ni, c0, nj, stream);
    case P_FP8: return launch_rect_p<P_FP8>(tile, C, N, n_spectra, spec, lay, scale2, out, first_call, r0, ni, c0, nj, stream);
    case P_INT8: return launch_rect_p<P_INT8>(tile, C, N, n_spectra, spec, lay, scale2, out, first_call, r0, ni, c0, nj, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_xengine(int prec, int tile, int C, int N, int n_spectra, const void *spec, SpecLayout lay,
                          const float *scale2, void *acc, const void *acc_in, int first_call, hipStream_t stream,
                          const int *zflag) {
#define CORR_X_ARGS tile, C, N, n_spectra, spec, lay, scale2, acc, acc_in, first_call, zflag, stream
    switch (prec) {
    case P_FP32: return launch_xp<P_FP32>(CORR_X_ARGS);
    case P_FP16: return launch_xp<P_FP16>(CORR_X_ARGS);
    case P_FP8: return launch_xp<P_FP8>(CORR_X_ARGS);
    case P_INT8: return launch_xp<P_INT8>(CORR_X_ARGS);
#undef CORR_X_ARGS
    default: return hipErrorInvalidValue;
    }
}

template <int PREC, int TILE>
hipError_t launch_batched_t(const XQueue *d_plan, const XDesc *d_desc, unsigned int *counter, int grid,
                            hipStream_t stream) {
    hipLaunchKernelGGL((xengine_batched_kernel<PREC, TILE>), dim3(grid), dim3(WaveGrid<TILE>::THREADS), 0, stream, d_plan, d_desc,
                       counter);
    return hipGetLastError();
}

template <int TILE>
hipError_t launch_batched_p(int prec, const XQueue *d_plan, const XDesc *d_desc, unsigned int *counter, int grid,
                            hipStream_t stream) {
    switch (prec) {
    case P_FP32: return launch_batched_t<P_FP32, TILE>(d_plan, d_desc, counter, grid, stream);
    case P_FP16: return launch_batched_t<P_FP16, TILE>(d_plan, d_desc, counter, grid, stream);
    case P_FP8: return launch_batched_t<P_FP8, TILE>(d_plan, d_desc, counter, grid, stream);
    case P_INT8: return launch_batched_t<P_INT8, TILE>(d_plan, d_desc, counter, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_xengine_batched(int prec, const XQueue *d_plan, const XDesc *d_desc, int launch_group,
                                  unsigned int *counters, int num_cus, hipStream_t stream) {
    if (num_cus <= 0 || (launch_group & ~3)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(2 * kXcds), 0, stream, counters);
    hipError_t e = hipGetLastError();
    // 128-input blocks first (the larger items), two workgroups per CU; then
    // 64-input blocks, four workgroups per CU.
    // (grids rounded to a multiple of the XCD count, as the kernel assumes)
    const int g128 = std::max(kXcds, 2 * num_cus / kXcds * kXcds), g64 = std::max(kXcds, 4 * num_cus / kXcds * kXcds);
    if (e == hipSuccess && (launch_group & 2))
        e = launch_batched_p<128>(prec, d_plan + 1, d_desc, counters + kXcds * kCounterStride, g128, stream);
    if (e == hipSuccess && (launch_group & 1))
        e = launch_batched_p<64>(prec, d_plan, d_desc, counters, g64, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(256), 0, stream, d_plan, d_desc);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_set_flag(int *flag, int v, hipStream_t stream) {
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, stream, flag, v);
    return hipGetLastError();
}

}  // namespace corr
