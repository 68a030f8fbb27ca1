// Internal declarations shared by the C-ABI layer and the HIP kernels.
//
// Spectra buffer layout (device, library-owned), "time-blocked planar": the
// 128-byte row of (channel k, time block tb, input p) -- plane 0 (real) then
// plane 1 (imaginary), TB spectra each, 64 bytes per plane -- sits at
//
//   spec + k * ks + tb * ts + p * 128
//
// with one of two stride pairs (SpecLayout, chosen per handle):
//   channel-major    [k][tb][p]: ts = N * 128, ks = n_tb_cap * N * 128 + pad
//   time-block-major [tb][k][p]: ks = N * 128 + pad, ts = C * ks
// Either way the rows of every input for one channel and one time block are
// one contiguous run of N * 128 bytes.  Time-block-major keeps the rows one
// F-engine workgroup writes (one input, every channel, one time block) within
// C * ks bytes however long the integration.  An X-engine tile of 128 inputs reads a
// contiguous 16 KB slab per time block, and each MFMA fragment (a row's K
// consecutive spectra of one plane) is a 16-byte vector.  Entries of the last
// time block beyond the valid spectra are zero, so every block can be
// correlated whole (zero spectra add nothing to Eq. 2).
//
// Accumulator layout (device, library-owned): acc[k][b], b = i(i+1)/2 + j for
// j <= i, each entry an (re, im) pair of float32 (float forms) or int32 (int8),
// i.e. the default dump layout, so a default dump is a plain copy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace corr {

enum Prec : int { P_FP32 = 0, P_FP16 = 1, P_FP8 = 2, P_INT8 = 3 };

// Bytes per (input, plane) row of one time block.
constexpr int kRowBytes = 64;
// Bytes added after each channel's slab of a time block.  Without it the
// channel stride is a power of two for power-of-two N and the F-engine's
// transposing stores (one per channel) all land in the same HBM channel.
constexpr int kChannelPad = 256;

struct SpecLayout {
    int64_t ks;                       // bytes between channels
    int64_t ts;                       // bytes between time blocks
};
// Measured on the MI355X: time-block-major is faster for the larger spectra
// buffers and for many inputs (2048 channels x 512 inputs x 2048 spectra:
// int8 F-engine 12.2 -> 9.3 ms; 4096 x 1024 x 1024 FP8: 28.7 -> 18.1 ms;
// 128 channels x 2048 inputs: F 0.61 -> 0.55 ms, X 1.37 -> 1.26 ms), and
// slower for the 1024 x 256 x 1000 case (FP32 F-engine 1.13 -> 1.47 ms).
inline bool default_tb_major(int C, int N, int elem) { return N >= 512 || C >= 2048 || C * elem < 1024; }
inline SpecLayout spec_layout_of(int C, int N, int n_tb_cap, bool tb_major) {
    const int64_t row = (int64_t)N * 2 * kRowBytes;
    if (tb_major) return {row + kChannelPad, (int64_t)C * (row + kChannelPad)};
    return {(int64_t)n_tb_cap * row + kChannelPad, row};
}
inline SpecLayout spec_layout(int C, int N, int n_tb_cap, int elem) {
    return spec_layout_of(C, N, n_tb_cap, default_tb_major(C, N, elem));
}
// Bytes of the spectra buffer: every row of n_tb_cap time blocks, plus
// padding, in whichever of the two orders needs more (a handle can switch).
inline int64_t spec_buffer_bytes(int C, int N, int n_tb_cap, int elem) {
    (void)elem;
    int64_t most = 0;
    for (int o = 0; o < 2; ++o) {
        const SpecLayout l = spec_layout_of(C, N, n_tb_cap, o == 1);
        const int64_t a = (int64_t)(C - 1) * l.ks + (int64_t)(n_tb_cap - 1) * l.ts + (int64_t)N * 2 * kRowBytes;
        most = a + kChannelPad > most ? a + kChannelPad : most;
    }
    return most;
}

inline int elem_bytes(int prec) { return prec == P_FP32 ? 4 : (prec == P_FP16 ? 2 : 1); }

// From kGatherMinC channels on, an F-engine workgroup holds too few spectra
// to write useful pieces of the 64-byte rows (4 bytes of each at 2048
// channels), and those scattered stores cap the kernel at 1-2.5 TB/s.  There
// the F-engine runs in chunks: each chunk's spectra go to a scratch buffer in
// the workgroups' natural order, contiguous per workgroup, and a gather
// kernel moves them into the rows.  Scratch bytes per (input, time block):
// C * 128.  kGatherScratchCap bounds the per-handle buffer (smaller chunks
// measured slower: each chunk adds two kernel tails, and even 32 MB chunks
// were not read back from the memory-side cache any faster).
constexpr int kGatherMinC = 2048;
constexpr int64_t kGatherScratchCap = (int64_t)1 << 30;
struct FScratch {
    void *buf;                        // device, library-owned; null below kGatherMinC
    int64_t bytes;
};
inline int64_t gather_scratch_bytes(int C, int N, int n_tb_cap) {
    if (C < kGatherMinC) return 0;
    const int64_t unit = (int64_t)C * 2 * kRowBytes;
    const int64_t all = unit * N * n_tb_cap;
    return all < kGatherScratchCap ? all : (kGatherScratchCap / unit) * unit;
}
// Spectra per time block.
inline int time_block(int prec) { return kRowBytes / elem_bytes(prec); }

// ---- launch entry points (each returns the launch's hipError_t) ----------

// F-engine: C-point FFTs of n_spectra blocks per input, requantised into the
// time-blocked planar spectra buffer.  Spectra in [n_spectra, n_tb*TB) of the
// last block are written as zeros.  inv_scale: C floats, never null.  The
// spectra land from time block first_tb of the buffer on.
// From kGatherMinC channels on the call runs in chunks through scr (see
// FScratch), one F-engine and one gather launch per chunk.
hipError_t launch_fengine(int prec, int C, int N, const float2 *volts, int64_t ld,
                          int n_spectra, const float *inv_scale, const float2 *twiddle,
                          void *spec, SpecLayout lay, FScratch scr, int first_tb, hipStream_t stream);

// F-engine on int8 real samples (Section 5): block a of row p is the 2C bytes
// samples[p*ld + a*2C ..]; channels k < C of its length-2C DFT.  twiddle2n[k]
// = exp(-j pi k / C), k < C.  ld even.
hipError_t launch_fengine_real8(int prec, int C, int N, const int8_t *samples, int64_t ld, int n_spectra,
                                const float *inv_scale, const float2 *twiddle, const float2 *twiddle2n,
                                void *spec, SpecLayout lay, FScratch scr, int first_tb, hipStream_t stream);

// X-engine: accumulate Eq. 2 over the first n_spectra spectra of the spectra
// buffer into acc (spectra past n_spectra in the last time block are masked to
// zero), with square blocks of `tile` (64 or 128) inputs.  scale2 (float
// forms, may be null = 1): per-channel s_k^2 applied to the integrated
// products.  first_call = 1 writes instead of read-modify-write; so does a
// set device flag *zflag (zflag may be null).  The sums so far are read from
// acc_in (acc itself, or the accumulators when acc is a dump destination in
// the accumulator layout).
hipError_t launch_xengine(int prec, int tile, int C, int N, int n_spectra, const void *spec, SpecLayout lay,
                          const float *scale2, void *acc, const void *acc_in, int first_call, hipStream_t stream,
                          const int *zflag = nullptr);

// Write v to the device int *flag (a kernel, so graphs replay it).
hipError_t launch_set_flag(int *flag, int v, hipStream_t stream);

// Rectangle X-engine: rows [r0, r0 + ni) against columns [c0, c0 + nj) of the
// held spectra (disjoint ranges), into out [C][ni][nj] (re, im) pairs, written
// when first_call, else added to.
hipError_t launch_xengine_rect(int prec, int tile, int C, int N, int n_spectra, const void *spec, SpecLayout lay,
                               const float *scale2, void *out, int first_call, int r0, int ni, int c0, int nj,
                               hipStream_t stream);

// One sub-array of a batched X-engine launch.  Items [item_begin,
// item_begin + C * n_tiles) are (channel, block) pairs of this sub-array.
// Accelerator complex dies (XCDs), each with its own L2; workgroups are
// dispatched to them round-robin by workgroup index.
constexpr int kXcds = 8;
// Work counters of the batched X-engine sit kCounterStride words apart (256
// bytes), one per cache line; 2 x 8 of them.
constexpr int kCounterStride = 64;

struct XDesc {
    const uint8_t *spec;
    void *acc;
    const float *scale2;
    int *zflag;                       // the sub-array's "zero since reset" flag (device)
    int64_t k_stride;                 // SpecLayout::ks
    int64_t tb_stride;                // SpecLayout::ts
    int64_t B;
    int64_t qbegin[kXcds];            // offset of this sub-array's items in each XCD's queue
    int C, N, n_tb, tv, tile, n_tiles, first_call, pad;
};

// Work plan of one block-size group, resident in device memory beside the
// descriptors it indexes (so a kernel never pairs queue lengths from one
// upload with descriptors from another).
struct XQueue {
    int64_t qlen[kXcds];              // items in each XCD's queue
    int n_desc;                       // descriptors of the group
    int desc_offset;                  // index of the group's first descriptor
};

// Persistent X-engine over sub-arrays in two groups by block size (plan[0]:
// 64-input blocks, plan[1]: 128-input blocks; descriptors of each group sorted
// by item cost, largest first).  XCD x's queue holds channels
// [x C/8, (x+1) C/8) of every sub-array of the group, in descriptor order.
// Workgroups take items from their own XCD's queue, then from the others,
// through per-queue atomic counters.  A 16-thread kernel zeroes the 2 x 8 counters
// (2 * kXcds * kCounterStride words), then one persistent launch per group in
// launch_group (bit 0: 64-input, bit 1: 128-input) runs at that block size's
// occupancy, and a last one-workgroup kernel clears the zero flag of every
// sub-array in the plan (an item whose flag is set writes its sums instead of
// adding to the accumulators).
hipError_t launch_xengine_batched(int prec, const XQueue *d_plan, const XDesc *d_desc, int launch_group,
                                  unsigned int *counters, int num_cus, hipStream_t stream);

// Public [A][C][N][2] spectra <-> internal layout (ingest zero-fills the tail
// of the last time block).
hipError_t launch_ingest(int prec, int C, int N, int n_spectra, SpecLayout lay, const void *src,
                         void *spec, hipStream_t stream);
hipError_t launch_export(int prec, int C, int N, int n_spectra, SpecLayout lay, const void *spec,
                         void *dst, hipStream_t stream);
// Ingest of channels [k0, k0 + nk) of public spectra with C channels into held
// channels [0, nk) of spec (laid out by lay).
hipError_t launch_ingest_channels(int prec, int C, int k0, int nk, int N, int n_spectra, SpecLayout lay,
                                  const void *src, void *spec, hipStream_t stream);

// Dump conversion from the lower-triangle channel-major accumulators into a
// layout (0 lower, 1 upper, 2 full) and order (0 chan-major, 1 baseline-major).
// Entries are 8-byte (re, im) pairs; is_int selects int32 negation for the
// conjugate of mirrored products.  A set device flag *zflag (zflag may be
// null) means the accumulators are logically zero: zeros are written.
hipError_t launch_dump_convert(int C, int N, int layout, int order, int is_int,
                               const void *acc, void *dst, hipStream_t stream, const int *zflag = nullptr);

// dst = acc (n_words 32-bit words), or zeros when *zflag is set.
hipError_t launch_dump_copy(const void *acc, void *dst, int64_t n_words, const int *zflag, hipStream_t stream);

// s_k^2 = 1 / inv_s[k]^2 (or 1 when inv_s is null) into scale2[C].
hipError_t launch_scale2(int C, const float *inv_scale, float *scale2, hipStream_t stream);

// Fill n 32-bit words with zero (a kernel, not a memset node, so the call is
// safe inside captured graphs).
hipError_t launch_zero(void *p, int64_t n_words, hipStream_t stream);

}  // namespace corr
