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
// Tiling.  A workgroup (256 threads, 4 waves) owns a 128x128 block (rows I,
// columns J <= I) of one channel; each wave a 64x64 quarter as 2x2 MFMA
// 32x32 blocks with separate real and imaginary accumulators.  On diagonal
// blocks the wave above the diagonal idles and the diagonal waves skip their
// upper 32x32 block.  The K loop walks time blocks: each stage copies the
// rows' contiguous 16 KB slab (128 inputs x 2 planes x 64 bytes) for I and J
// from global memory into padded LDS rows (144-byte stride, conflict-free
// 16-byte fragment reads), double-buffered with one barrier per stage.
// Every lane reads 32 bytes per (fragment, plane) per stage, which is one K
// step for FP8 (32x32x64), two for int8 (32x32x32) and FP16 (32x32x16), and
// eight for FP32 (32x32x2).  Because the same K assignment is used for both
// operands, the spectrum-to-slot order inside a stage does not matter.
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

constexpr int kXThreads = 256;
constexpr int kRowStride = 144;                   // 2 planes x 64 B + 16 B pad
// LDS bytes of one operand slab and of one stage (two slabs) for a tile size.
constexpr int op_bytes(int tile) { return tile * kRowStride; }
constexpr int stage_bytes(int tile) { return 2 * op_bytes(tile); }
constexpr int kMaxStageBytes = stage_bytes(128);

// Per-precision fragment type and MFMA step.  A lane owns 32 bytes of each
// (row, plane) per time block, read as KS fragments of FB bytes; each
// fragment feeds NSUB MFMAs (sub-element e of the fragment).
template <int PREC> struct XT;

template <> struct XT<P_FP32> {
    using Acc = f32x16;
    using Frag = f32x4;   // 4 spectra; 16-byte LDS reads are bank-conflict free
    static constexpr int KS = 2, FB = 16, NSUB = 4;
    static __device__ __forceinline__ Frag load(const uint8_t *p) { return *reinterpret_cast<const f32x4 *>(p); }
    static __device__ __forceinline__ Frag neg(Frag b) { return -b; }
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int e) {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], c, 0, 0, 0);
    }
};

template <> struct XT<P_FP16> {
    using Acc = f32x16;
    using Frag = i32x4;
    static constexpr int KS = 2, FB = 16, NSUB = 1;
    static __device__ __forceinline__ Frag load(const uint8_t *p) { return *reinterpret_cast<const i32x4 *>(p); }
    static __device__ __forceinline__ Frag neg(Frag b) {
        return Frag{b[0] ^ (int)0x80008000u, b[1] ^ (int)0x80008000u, b[2] ^ (int)0x80008000u,
                    b[3] ^ (int)0x80008000u};
    }
    static __device__ __forceinline__ f16x8 h8(Frag x) { return __builtin_bit_cast(f16x8, x); }
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(h8(a), h8(b), c, 0, 0, 0);
    }
};

template <> struct XT<P_INT8> {
    using Acc = i32x16;
    using Frag = i32x4;
    static constexpr int KS = 2, FB = 16, NSUB = 1;
    static __device__ __forceinline__ Frag load(const uint8_t *p) { return *reinterpret_cast<const i32x4 *>(p); }
    // Byte-wise 0 - b without borrows between bytes.
    static __device__ __forceinline__ int neg4(int v) {
        const uint32_t x = (uint32_t)v;
        return (int)((0x80808080u - (x & 0x7f7f7f7fu)) ^ (~x & 0x80808080u));
    }
    static __device__ __forceinline__ Frag neg(Frag b) { return Frag{neg4(b[0]), neg4(b[1]), neg4(b[2]), neg4(b[3])}; }
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int) {
        c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
    }
};

template <> struct XT<P_FP8> {
    using Acc = f32x16;
    using Frag = i32x8;
    static constexpr int KS = 1, FB = 32, NSUB = 1;
    static __device__ __forceinline__ Frag load(const uint8_t *p) {
        const i32x4 a = *reinterpret_cast<const i32x4 *>(p);
        const i32x4 b = *reinterpret_cast<const i32x4 *>(p + 16);
        return Frag{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    }
    static __device__ __forceinline__ Frag neg(Frag b) {
        Frag r;
#pragma unroll
        for (int t = 0; t < 8; ++t) r[t] = b[t] ^ (int)0x80808080u;
        return r;
    }
    // Format code 0 = FP8 E4M3 for both operands; E8M0 scale 127 = 2^0.
    static __device__ __forceinline__ void mfma(Acc &c, const Frag &a, const Frag &b, int) {
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
    }
};

// One time block of a wave's quarter (FS x FS blocks of 32x32; FS = 2 for
// 128-input tiles, 1 for 64-input tiles): KS fragment reads per (row or column
// block, plane), NSUB MFMAs per fragment, four real products per 32x32 block
// (Re += Ar Br + Ai Bi, Im += Ar Bi + Ai (-Br)), issued across the column
// blocks so dependent MFMAs are apart.  SKIP_UPPER (FS = 2 only): a diagonal
// wave leaves out its upper 32x32 block (rows 0-31, columns 32-63).
template <int PREC, int FS, bool SKIP_UPPER, typename Acc>
__device__ __forceinline__ void wave_block(Acc (&re)[FS][FS], Acc (&im)[FS][FS], const uint8_t *pa,
                                           const uint8_t *pb) {
    using X = XT<PREC>;
#pragma unroll
    for (int s = 0; s < X::KS; ++s) {
        typename X::Frag b[FS][2], nb[FS];
#pragma unroll
        for (int g = 0; g < FS; ++g) {
            b[g][0] = X::load(pb + g * 32 * kRowStride + s * X::FB);
            b[g][1] = X::load(pb + g * 32 * kRowStride + kRowBytes + s * X::FB);
            nb[g] = X::neg(b[g][0]);
        }
#pragma unroll
        for (int f = 0; f < FS; ++f) {
            const typename X::Frag ar = X::load(pa + f * 32 * kRowStride + s * X::FB);
            const typename X::Frag ai = X::load(pa + f * 32 * kRowStride + kRowBytes + s * X::FB);
#pragma unroll
            for (int e = 0; e < X::NSUB; ++e) {
#pragma unroll
                for (int g = 0; g < FS; ++g)
                    if (!(SKIP_UPPER && f < g)) X::mfma(re[f][g], ar, b[g][0], e);    // + xr_i xr_j
#pragma unroll
                for (int g = 0; g < FS; ++g)
                    if (!(SKIP_UPPER && f < g)) X::mfma(im[f][g], ar, b[g][1], e);    // + xr_i xi_j
#pragma unroll
                for (int g = 0; g < FS; ++g)
                    if (!(SKIP_UPPER && f < g)) X::mfma(re[f][g], ai, b[g][1], e);    // + xi_i xi_j
#pragma unroll
                for (int g = 0; g < FS; ++g)
                    if (!(SKIP_UPPER && f < g)) X::mfma(im[f][g], ai, nb[g], e);      // - xi_i xr_j
            }
        }
    }
}

// The whole K loop and epilogue of one TILE x TILE block of channel k, rows
// I0.., columns J0...  Both operand slabs are always staged (a diagonal block
// stages the same rows twice) so the staging code has no branches between
// its global loads.  4 waves, each owning a (TILE/2) x (TILE/2) quarter.
template <int PREC, int TILE>
__device__ __forceinline__ void tile(uint8_t *smem, const uint8_t *__restrict__ base_k, int N, int n_tb, int tv,
                                     int I0, int J0, int k, const float *__restrict__ scale2,
                                     void *__restrict__ acc_out, int64_t B, int first_call, int tid) {
    using Acc = typename XT<PREC>::Acc;
    constexpr int ES = PREC == P_FP32 ? 4 : (PREC == P_FP16 ? 2 : 1);
    constexpr int TB = kRowBytes / ES;
    constexpr int QS = TILE / 2;                        // rows of a wave's quarter
    constexpr int FS = QS / 32;                         // 32x32 blocks per quarter side
    constexpr int U = TILE / 32;                        // 16-byte chunks per thread per slab
    constexpr int OPB = op_bytes(TILE), STB = stage_bytes(TILE);
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = wave >> 1, wj = wave & 1;
    const int m = lane & 31, h = lane >> 5;
    const bool diag = I0 == J0;
    const bool active = !(diag && wj > wi);
    const bool dwave = FS > 1 && diag && wi == wj;      // skip the upper 32x32 block

    // Global -> register staging of one time block.  The loads are issued
    // unconditionally (rows past N read row N-1) and nothing inspects the
    // registers until store_stage, which runs after the block's MFMAs, so the
    // loads stay in flight during the compute.  store_stage zeroes rows past N
    // and, in the last time block, spectra past the valid count.
    uint4 st[2 * U];
    gu8 *const gbase = (gu8 *)base_k;
    auto load_stage = [&](int tb) {
        gu8 *blk = gbase + (int64_t)tb * N * (2 * kRowBytes);
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = tid + kXThreads * u;
                const int row = c >> 3, col = c & 7;
                const int pr = min((o ? J0 : I0) + row, N - 1);
                const u32x4 q = *(gu4 *)(blk + (int64_t)pr * (2 * kRowBytes) + col * 16);
                st[U * o + u] = make_uint4(q.x, q.y, q.z, q.w);
            }
    };
    auto store_stage = [&](int buf, int tb) {
        uint8_t *sm = smem + buf * STB;
        const bool tail = tb == n_tb - 1 && tv < TB;
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = tid + kXThreads * u;
                const int row = c >> 3, col = c & 7;
                uint4 v = st[U * o + u];
                if ((o ? J0 : I0) + row >= N) v = make_uint4(0, 0, 0, 0);
                if (tail) {
                    // zero the spectra past the valid count in the last time block
                    const int off = (col & 3) * 16;
                    uint32_t *wd = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        uint32_t msk = 0;
#pragma unroll
                        for (int bb = 0; bb < 4; ++bb)
                            if ((off + 4 * d + bb) / ES < tv) msk |= 0xffu << (8 * bb);
                        wd[d] &= msk;
                    }
                }
                *reinterpret_cast<uint4 *>(sm + o * OPB + row * kRowStride + col * 16) = v;
            }
    };

    Acc re[FS][FS], im[FS][FS];
#pragma unroll
    for (int f = 0; f < FS; ++f)
#pragma unroll
        for (int g = 0; g < FS; ++g) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                re[f][g][r] = 0;
                im[f][g][r] = 0;
            }
        }

    load_stage(0);
    store_stage(0, 0);
    __syncthreads();
    for (int tb = 0; tb < n_tb; ++tb) {
        const bool more = tb + 1 < n_tb;
        if (more) load_stage(tb + 1);
        if (active) {
            const uint8_t *sI = smem + (tb & 1) * STB;
            const uint8_t *sJ = sI + OPB;
            const uint8_t *pa = sI + (wi * QS + m) * kRowStride + h * 32;
            const uint8_t *pb = sJ + (wj * QS + m) * kRowStride + h * 32;
            // one uniform branch per block keeps the MFMA stream branch-free
            if (dwave)
                wave_block<PREC, FS, true>(re, im, pa, pb);
            else
                wave_block<PREC, FS, false>(re, im, pa, pb);
        }
        if (more) store_stage((tb + 1) & 1, tb + 1);
        __syncthreads();
    }
    if (!active) return;

    // Epilogue: element r of a 32x32 block is (row 8(r/4) + 4h + r%4, column m).
    // All of a block's accumulator reads are issued before any write; elements
    // outside the triangle or past N read a valid address and are not written.
    using E = typename std::conditional<PREC == P_INT8, int, float>::type;
    typedef E T2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) T2 gT2;
    gT2 *out = (gT2 *)acc_out + (int64_t)k * B;
    const float s2 = (PREC != P_INT8 && scale2) ? ((gf32 *)scale2)[k] : 1.0f;
#pragma unroll
    for (int f = 0; f < FS; ++f)
#pragma unroll
        for (int g = 0; g < FS; ++g) {
            if (dwave && f < g) continue;
            const int j = J0 + wj * QS + g * 32 + m;
            int64_t idx[16];
            uint32_t ok = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = I0 + wi * QS + f * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const bool in = i < N && j <= i;
                ok |= (uint32_t)in << r;
                idx[r] = in ? (int64_t)i * (i + 1) / 2 + j : 0;
            }
            T2 old[16];
            if (!first_call) {
#pragma unroll
                for (int r = 0; r < 16; ++r) old[r] = out[idx[r]];
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = I0 + wi * QS + f * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                T2 v;
                if constexpr (PREC == P_INT8) {
                    v = T2{re[f][g][r], i == j ? 0 : im[f][g][r]};
                } else {
                    v = T2{re[f][g][r] * s2, i == j ? 0.0f : im[f][g][r] * s2};
                }
                if (!first_call) {
                    v.x += old[r].x;
                    v.y += old[r].y;
                }
                if ((ok >> r) & 1u) out[idx[r]] = v;
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

template <int PREC, int TILE>
__global__ __launch_bounds__(kXThreads) __attribute__((amdgpu_waves_per_eu(2))) void xengine_kernel(
    const uint8_t *__restrict__ spec, int N, int n_tiles, int n_work, int n_tb, int tv,
    int64_t k_stride, const float *__restrict__ scale2, void *__restrict__ acc_out, int64_t B,
    int first_call) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[2 * stage_bytes(TILE)];
    const int per = (n_work + 7) / 8;
    const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= n_work) return;
    const int k = w / n_tiles;
    int bi, bj;
    tri_block(w % n_tiles, bi, bj);
    tile<PREC, TILE>(smem, spec + (int64_t)k * k_stride, N, n_tb, tv, bi * TILE, bj * TILE, k, scale2, acc_out,
                     B, first_call, threadIdx.x);
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
__global__ __launch_bounds__(kXThreads) __attribute__((amdgpu_waves_per_eu(TILE == 64 ? 4 : 2))) void xengine_batched_kernel(
    const XQueue *__restrict__ plan, const XDesc *__restrict__ all_desc, unsigned int *__restrict__ counter) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[2 * stage_bytes(TILE)];
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
        while (item < qlen) {
            // take the next ticket now; its latency overlaps this item's loads
            unsigned int next = 0;
            if (tid == 0) next = atomicAdd(cnt, 1u);
            int lo = 0, hi = n_desc - 1;                // last descriptor with qbegin[x] <= item
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (desc[mid].qbegin[x] <= item) lo = mid; else hi = mid - 1;
            }
            const XDesc &d = desc[lo];
            const int64_t local = item - d.qbegin[x];
            const int k = x * d.C / kXcds + (int)(local / d.n_tiles);
            int bi, bj;
            tri_block((int)(local % d.n_tiles), bi, bj);
            // an opaque copy of the thread index keeps the block body's
            // per-lane address arithmetic inside the loop instead of live
            // across it (which cost registers and occupancy)
            int t = tid;
            asm volatile("" : "+v"(t));
            tile<PREC, TILE>(smem, d.spec + (int64_t)k * d.k_stride, d.N, d.n_tb, d.tv, bi * TILE, bj * TILE, k,
                             d.scale2, d.acc, d.B, d.first_call, t);
            if (tid == 0) s_item = next;
            __syncthreads();                            // also: every wave is done with smem
            item = (unsigned int)__builtin_amdgcn_readfirstlane((int)s_item);
            __syncthreads();
        }
    }
}

__global__ void reset_counters_kernel(unsigned int *counter) { counter[threadIdx.x * kCounterStride] = 0u; }

template <int PREC, int TILE>
hipError_t launch_x(int C, int N, int n_spectra, int n_tb_cap, const void *spec, const float *scale2,
                    void *acc, int first_call, hipStream_t stream) {
    const int TB = time_block(PREC);
    const int n_tb = (n_spectra + TB - 1) / TB;
    const int tv = n_spectra - (n_tb - 1) * TB;
    const int n_blk = (N + TILE - 1) / TILE;
    const int n_tiles = n_blk * (n_blk + 1) / 2;
    const int64_t n_work = (int64_t)C * n_tiles;
    if (n_tb <= 0 || n_work <= 0 || n_work > ((int64_t)1 << 30)) return hipErrorInvalidValue;
    const int grid = (int)((n_work + 7) / 8) * 8;
    const int64_t k_stride = channel_stride(n_tb_cap, N);
    const int64_t B = (int64_t)N * (N + 1) / 2;
    hipLaunchKernelGGL((xengine_kernel<PREC, TILE>), dim3(grid), dim3(kXThreads), 0, stream,
                       static_cast<const uint8_t *>(spec), N, n_tiles, (int)n_work, n_tb, tv, k_stride,
                       scale2, acc, B, first_call);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_xp(int tile, int C, int N, int n_spectra, int n_tb_cap, const void *spec, const float *scale2,
                     void *acc, int first_call, hipStream_t stream) {
    if (tile == 64) return launch_x<PREC, 64>(C, N, n_spectra, n_tb_cap, spec, scale2, acc, first_call, stream);
    if (tile == 128) return launch_x<PREC, 128>(C, N, n_spectra, n_tb_cap, spec, scale2, acc, first_call, stream);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_xengine(int prec, int tile, int C, int N, int n_spectra, int n_tb_cap, const void *spec,
                          const float *scale2, void *acc, int first_call, hipStream_t stream) {
    switch (prec) {
    case P_FP32: return launch_xp<P_FP32>(tile, C, N, n_spectra, n_tb_cap, spec, scale2, acc, first_call, stream);
    case P_FP16: return launch_xp<P_FP16>(tile, C, N, n_spectra, n_tb_cap, spec, scale2, acc, first_call, stream);
    case P_FP8: return launch_xp<P_FP8>(tile, C, N, n_spectra, n_tb_cap, spec, scale2, acc, first_call, stream);
    case P_INT8: return launch_xp<P_INT8>(tile, C, N, n_spectra, n_tb_cap, spec, scale2, acc, first_call, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int PREC, int TILE>
hipError_t launch_batched_t(const XQueue *d_plan, const XDesc *d_desc, unsigned int *counter, int grid,
                            hipStream_t stream) {
    hipLaunchKernelGGL((xengine_batched_kernel<PREC, TILE>), dim3(grid), dim3(kXThreads), 0, stream, d_plan, d_desc,
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
    return e;
}

}  // namespace corr
