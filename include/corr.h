/*
 * corr.h -- C ABI of the MI355X FX-correlator hot path.
 *
 * The library implements, on one gfx950 GPU, the two engines of an FX
 * correlator (Wang & Harris, "Scaling Radio Astronomy Signal Correlation on
 * Heterogeneous Supercomputers Using Various Data Distribution
 * Methodologies", Exp. Astron. 2013):
 *
 *   F-engine (Section 2, Eq. 1): every input stream is cut into consecutive,
 *     non-overlapping blocks of C samples and each block is transformed with a
 *     forward, unnormalised C-point complex DFT, S[k] = sum_n s[n] e^{-j 2 pi k n / C},
 *     giving C channels in natural order.  No window, filter bank or fringe
 *     rotation (the paper's F-engine carries none, Section 5).
 *
 *   X-engine (Section 2, Eq. 2): for every channel k and every pair (i, j) of
 *     the triangle of non-redundant input pairs, autos included (Section 4),
 *     C_ij[k] = sum_a conj(S_{a,i}[k]) S_{a,j}[k] -- conjugate on the FIRST
 *     index -- summed (not averaged) over the spectra a of the integration.
 *
 * An "input" is one station-polarisation stream: input p = station*n_pols + pol
 * (a stream carries one polarisation of one antenna, Section 3).  N inputs give
 * N(N+1)/2 products per channel.
 *
 * Conventions for every function:
 *   - Every function returns a corr_status; nothing throws across the ABI.
 *   - Output parameters are written only on CORR_OK.
 *   - Argument validation runs on the CPU before any HIP call, so invalid
 *     arguments never touch the device.
 *   - All device work is enqueued on the HIP stream given to corr_create and
 *     is asynchronous, except where a function says it synchronises.  Caller
 *     buffers must stay valid until that work completes.
 *   - Pointers named d_* are device pointers; the caller owns them.  The
 *     library owns the handle, its spectra buffer and its accumulators.
 *   - A handle must not be used from two threads at once.
 */
#ifndef CORR_H
#define CORR_H

#include <stdint.h>

#if defined(__GNUC__)
#define CORR_API __attribute__((visibility("default")))
#else
#define CORR_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct corr_ctx *corr_handle;

typedef enum {
    CORR_OK = 0,
    CORR_E_INVALID_ARG = 1, /* a null pointer, out-of-range value or misaligned buffer   */
    CORR_E_UNSUPPORTED = 2, /* a well-formed request outside what the library implements */
    CORR_E_NOMEM = 3,       /* the plan does not fit the device memory budget            */
    CORR_E_OVERFLOW = 4,    /* the int8 integration could overflow its int32 accumulators */
    CORR_E_STATE = 5,       /* calls made out of order (e.g. X before any F)             */
    CORR_E_HIP = 6          /* a HIP runtime error; corr_last_error() holds its text     */
} corr_status;

/* Arithmetic forms of the X-engine input (the F-engine requantises into it).
 *   CORR_FP32     : float32 spectra, float32 accumulation.
 *   CORR_FP16     : IEEE binary16 spectra (round half to even, saturating at
 *                   +-65504), float32 accumulation.
 *   CORR_FP8_E4M3 : OCP FP8 E4M3 spectra (round half to even, saturating at
 *                   +-448, no infinities), float32 accumulation.
 *   CORR_INT8     : int8 spectra, round half to even, clamped to [-127, 127]
 *                   (the paper's inputs are 8-bit integers, Section 5), exact
 *                   int32 accumulation. */
typedef enum { CORR_FP32 = 0, CORR_FP16 = 1, CORR_FP8_E4M3 = 2, CORR_INT8 = 3 } corr_precision;

/* Layout of one channel's products in a dump.
 *   CORR_TRI_LOWER : rows i in [0,N), columns j <= i, b = i(i+1)/2 + j, value C_ij.
 *   CORR_TRI_UPPER : rows i, columns j >= i, b = i*N - i(i-1)/2 + (j - i), value C_ij.
 *   CORR_FULL      : all N*N products, b = i*N + j (C_ij = conj(C_ji)). */
typedef enum { CORR_TRI_LOWER = 0, CORR_TRI_UPPER = 1, CORR_FULL = 2 } corr_layout;

/* Order of a dump: channel-major [k][b] or baseline-major [b][k]. */
typedef enum { CORR_CHAN_MAJOR = 0, CORR_BASELINE_MAJOR = 1 } corr_order;

typedef struct {
    int32_t n_stations;      /* >= 1                                                     */
    int32_t n_pols;          /* 1 or 2; input p = station*n_pols + pol                    */
    int32_t n_channels;      /* C = FFT length = channel count; power of two, 16..8192   */
    int32_t n_integrate;     /* A of Eq. 2 for one X-engine call: the spectra the handle
                                holds (capacity of its spectra buffer), so the largest
                                n_spectra of one F- or X-engine call.  An integration
                                may span several X-engine calls (it ends at a dump with
                                reset), so it can be longer than n_integrate.           */
    int32_t precision;       /* corr_precision                                           */
    int32_t layout;          /* corr_layout used by corr_dump_visibilities               */
    int32_t order;           /* corr_order used by corr_dump_visibilities                */
    int32_t reserved;        /* must be 0                                                */
    uint64_t device_mem_cap; /* bytes the plan may use; 0 = the device's free memory     */
} corr_params;

/* Limits. */
#define CORR_MIN_CHANNELS 16
#define CORR_MAX_CHANNELS 8192
#define CORR_MAX_INPUTS 8192
/* Largest int8 integration whose worst case, 2*127^2 per spectrum, fits int32. */
#define CORR_INT8_MAX_INTEGRATE 66572

/* Number of products per channel: the triangle of non-redundant input pairs,
 * autos included (Section 4), N(N+1)/2 with N = n_stations*n_pols, each a
 * C_ij of Eq. 2; -1 on bad params. */
CORR_API int64_t corr_n_products(const corr_params *params);

/* Bytes one corr_dump_visibilities writes: products in the chosen layout x
 * channels x 8 (complex64 for float forms, an (re, im) int32 pair for int8);
 * -1 on bad params. */
CORR_API int64_t corr_visibility_bytes(const corr_params *params);

/* Bytes of n_spectra spectra in the public spectra layout (see corr_xengine);
 * -1 on bad params. */
CORR_API int64_t corr_spectra_bytes(const corr_params *params, int32_t n_spectra);

/*
 * Plan and allocate a correlator for the given shape.  Validates params
 * (CORR_E_INVALID_ARG / CORR_E_UNSUPPORTED), sizes the spectra buffer
 * (n_integrate spectra), the accumulators (C * N(N+1)/2 complex), the
 * twiddle tables and, from 2048 channels on, an F-engine scratch buffer
 * (C * 128 * N * ceil(n_integrate / time block) bytes, or 1 GiB rounded down
 * to whole C * 128-byte units if that is less).  It fails with CORR_E_NOMEM
 * when these exceed device_mem_cap (or the device's free memory when the cap
 * is 0): the failure mode of a GPU
 * that cannot hold all baselines of one FFT length (Section 3).  For
 * CORR_INT8, n_integrate above CORR_INT8_MAX_INTEGRATE is CORR_E_OVERFLOW.
 * hip_stream is a hipStream_t (NULL = the null stream); all later work of the
 * handle is enqueued on it.  Accumulators start at zero.  Launches no kernel.
 */
CORR_API corr_status corr_create(const corr_params *params, void *hip_stream, corr_handle *out);

/* Release the handle and its device memory (synchronises its stream).
 * A NULL handle is CORR_E_INVALID_ARG. */
CORR_API corr_status corr_destroy(corr_handle h);

/*
 * F-engine (Eq. 1) with the requantise epilogue of the handle's precision.
 *   d_volts     : complex64 (float re, im) voltages, [n_inputs][ld_samples];
 *                 spectrum a of input p is the DFT of samples
 *                 [a*C, (a+1)*C) of row p.  8-byte aligned.
 *   ld_samples  : row stride in complex samples, >= n_spectra*C.
 *   n_spectra   : 1 .. n_integrate spectra to channelise.
 *   d_inv_scale : float32 [C] per-channel scale inv_s[k]; each spectrum value
 *                 is multiplied by inv_s[k] before requantisation, and the
 *                 X-engine multiplies the integrated products by s_k^2 =
 *                 1/inv_s[k]^2 so that dumps are in voltage units (the int8
 *                 form dumps raw integer sums instead).  Required for
 *                 CORR_INT8; NULL means 1.0 for the other forms.
 * The spectra replace the handle's previous spectra.
 */
CORR_API corr_status corr_fengine(corr_handle h, const void *d_volts, int64_t ld_samples,
                         int32_t n_spectra, const float *d_inv_scale);

/*
 * F-engine on 8-bit real samples (Section 5: every test stream is 8-bit real
 * integers and the transform length is 256), with the same requantise
 * epilogue and the same held spectra as corr_fengine.
 *   d_samples   : int8 real samples, [n_inputs][ld_samples]; spectrum a of
 *                 input p is the length-2C DFT (Eq. 1 with 2C points) of
 *                 samples [a*2C, (a+1)*2C) of row p, of which channels
 *                 0 .. C-1 are kept (the Nyquist channel C is dropped), C the
 *                 handle's n_channels.  2-byte aligned.
 *   ld_samples  : row stride in samples (bytes), even, >= n_spectra*2C.
 *   n_spectra, d_inv_scale : as for corr_fengine.
 * The spectra replace the handle's previous spectra; corr_xengine then
 * correlates them as usual.
 */
CORR_API corr_status corr_fengine_real8(corr_handle h, const int8_t *d_samples, int64_t ld_samples,
                                        int32_t n_spectra, const float *d_inv_scale);

/*
 * The same two F-engines writing at an offset of the held spectra, so that an
 * integration (Eq. 2) longer than one batch of samples can be channelised in
 * pieces and correlated by one corr_xengine call, which reads and writes the
 * accumulators once instead of once per piece.
 *   first_spectrum : where the n_spectra new spectra go in the held set.  A
 *                    multiple of the time block (16 spectra for CORR_FP32, 32
 *                    for CORR_FP16, 64 for CORR_FP8_E4M3 and CORR_INT8);
 *                    first_spectrum + n_spectra <= n_integrate.  0 is the
 *                    plain call.  Above 0 the held spectra must come from an
 *                    F-engine and reach first_spectrum (no gap), else
 *                    CORR_E_STATE.  Afterwards the held set is
 *                    [0, first_spectrum + n_spectra).
 * Every piece of one held set must use the same d_inv_scale: the X-engine
 * rescales all held spectra with the last call's s_k^2.
 * The other arguments are as for corr_fengine / corr_fengine_real8; the data
 * read are samples [0, n_spectra*C) (resp. 2C) of each row of this call's
 * buffer.
 */
CORR_API corr_status corr_fengine_at(corr_handle h, const void *d_volts, int64_t ld_samples,
                                     int32_t n_spectra, const float *d_inv_scale, int32_t first_spectrum);
CORR_API corr_status corr_fengine_real8_at(corr_handle h, const int8_t *d_samples, int64_t ld_samples,
                                           int32_t n_spectra, const float *d_inv_scale,
                                           int32_t first_spectrum);

/*
 * X-engine (Eq. 2): add n_spectra spectra into the accumulators.
 *   d_spectra   : NULL = the first n_spectra spectra of the last corr_fengine
 *                 (n_spectra above that call's count is CORR_E_STATE); else
 *                 caller spectra in the public layout
 *                 [n_spectra][n_channels][n_inputs][2] of the precision's
 *                 element (float32, binary16, E4M3 byte or int8; re then im),
 *                 16-byte aligned, n_spectra <= n_integrate.  Caller spectra
 *                 overwrite the handle's spectra buffer.  CORR_INT8 caller
 *                 values are taken in [-127, 127]: -128 is read as -127 (the
 *                 same symmetric clamp as the F-engine's requantiser, which
 *                 keeps negation exact and the int32 bound below valid).
 *   d_inv_scale : with caller spectra of the FP16 / FP8 forms, the float32
 *                 per-channel inv_s[k] they were scaled with (NULL = 1.0);
 *                 must be NULL when d_spectra is NULL (the F-engine's scale
 *                 applies) and for CORR_FP32 / CORR_INT8.
 * For CORR_INT8, a running integration longer than CORR_INT8_MAX_INTEGRATE
 * spectra since the last reset is CORR_E_OVERFLOW (nothing is launched).
 */
CORR_API corr_status corr_xengine(corr_handle h, const void *d_spectra, int32_t n_spectra,
                         const float *d_inv_scale);

/*
 * F and X fused over time chunks (Eq. 1 then Eq. 2): the n_spectra spectra
 * of d_volts (as for corr_fengine) are channelised and correlated
 * chunk_spectra at a time -- the F-engine writes a chunk into the first
 * chunk_spectra slots of the held spectra and the X-engine adds it into the
 * accumulators right away -- so a chunk small enough stays in the
 * memory-side cache between the two (the paper keeps its F output close to
 * the X-engine and ships it packed, Section 6).  The result is that of one
 * corr_fengine + corr_xengine over the whole integration (bit for bit for
 * CORR_INT8; the float forms sum in another order), and n_spectra may exceed
 * n_integrate.  Afterwards the held spectra are the last chunk's.
 *   chunk_spectra : a multiple of the time block (16 FP32, 32 FP16, 64 FP8 /
 *                   int8 spectra), at most n_integrate.
 * Every chunk reads and writes the accumulators once more, which is why the
 * unfused corr_fengine + corr_xengine is the faster path on the configured
 * workloads.  Errors as corr_fengine and corr_xengine (CORR_E_STATE for batch
 * sub-arrays).
 */
CORR_API corr_status corr_fx(corr_handle h, const void *d_volts, int64_t ld_samples, int32_t n_spectra,
                             const float *d_inv_scale, int32_t chunk_spectra);

/*
 * The last X-engine call of an integration fused with its dump: as
 * corr_xengine, but the integrated visibilities (the accumulators' sums plus
 * this call's) are written straight to d_dst, in the dump's lower-triangle,
 * channel-major layout and units, instead of back into the accumulators, and
 * the integration is reset -- the same result as corr_xengine followed by
 * corr_dump_visibilities(h, d_dst, 1, 1), without the copy.
 *   d_dst : device pointer, 8-byte aligned, corr_visibility_bytes(params)
 *           bytes.
 * Handles whose layout is not CORR_TRI_LOWER / CORR_CHAN_MAJOR are
 * CORR_E_UNSUPPORTED; batch sub-array handles are CORR_E_STATE.  The other
 * arguments and errors are as for corr_xengine.
 */
CORR_API corr_status corr_xengine_dump(corr_handle h, const void *d_spectra, int32_t n_spectra,
                                       const float *d_inv_scale, void *d_dst);

/*
 * Dump (Eq. 2 integrated over the spectra since the last reset; Section 4's
 * triangle of non-redundant pairs, or the full matrix on request).
 * Write the integrated visibilities to dst in the handle's layout and order:
 * complex64 per product for the float forms (scaled to voltage units),
 * (re, im) int32 per product for CORR_INT8 (raw integer sums, exact).
 * dst holds corr_visibility_bytes(params) bytes; dst_on_device = 1 for a
 * device pointer (asynchronous), 0 for host memory (synchronises the stream).
 * reset = 1 zeroes the accumulators afterwards (a new integration starts);
 * reset = 0 keeps them, so further corr_xengine calls continue the same
 * integration (resume).
 */
CORR_API corr_status corr_dump_visibilities(corr_handle h, void *dst, int32_t dst_on_device, int32_t reset);

/*
 * Copy the spectra held by the handle -- the S[k] of Eq. 1 for each input and
 * spectrum after the requantise epilogue, i.e. exactly the values Eq. 2
 * correlates (the paper packs them into 8-bit integers before correlation,
 * Section 5) -- to dst in the public spectra
 * layout [n_spectra][n_channels][n_inputs][2] of the precision's element.
 * dst holds corr_spectra_bytes(params, n) bytes, n = spectra held.  With
 * dst_on_device = 0 the call synchronises the stream.  For checking and
 * debugging; not on the hot path.
 */
CORR_API corr_status corr_copy_spectra(corr_handle h, void *dst, int32_t dst_on_device);

/*
 * Cross-correlation of two disjoint input ranges: a rectangle of the
 * triangle of pairs, the product a node forms in the paper's space-division
 * models (Section 4), where one group of streams is correlated against
 * another.  For every channel k, rows i in [i0, i0 + ni) and columns j in
 * [j0, j0 + nj):
 *     R[k][i - i0][j - j0] = s_k^2 sum_a conj(S_a,i[k]) S_a,j[k]      (Eq. 2)
 * over the first n_spectra held spectra (the first index is conjugated, as in
 * corr_xengine; i0 > j0 gives entries of the lower triangle, i0 < j0 their
 * conjugates).  The ranges must not overlap (i0 + ni <= j0 or j0 + nj <= i0);
 * for a triangle use corr_xengine.  d_out: caller-owned device buffer of
 * C * ni * nj (re, im) pairs, float32 (int32 for CORR_INT8, unscaled), 8-byte
 * aligned, [C][ni][nj] row-major; accumulate = 0 writes it, 1 adds to it.  The
 * handle's accumulators and counters are not touched, so the library does not
 * track a running total across accumulate = 1 calls: for CORR_INT8 the caller
 * keeps the spectra summed into one d_out at or below CORR_INT8_MAX_INTEGRATE,
 * or its int32 entries can wrap.  Errors:
 * CORR_E_INVALID_ARG (ranges, overlap, pointer, flag), CORR_E_STATE (no or
 * too few spectra held), CORR_E_OVERFLOW (int8 over 66572 spectra in one call).
 */
CORR_API corr_status corr_xengine_rect(corr_handle h, int32_t i0, int32_t ni, int32_t j0, int32_t nj,
                                       int32_t n_spectra, void *d_out, int32_t accumulate);

/* Number of spectra currently held, and spectra integrated since the last reset. */
CORR_API corr_status corr_get_counts(corr_handle h, int32_t *n_held, int64_t *n_integrated);

/*
 * X-engine block size.  The triangle of each channel is covered by square
 * blocks of `tile` inputs (64 or 128); 0 selects a default unless
 * corr_autotune has chosen: 64 for FP32 and for N <= 64, else 128.  Larger blocks reuse each operand more; smaller ones
 * run more workgroups per CU and waste less on the diagonal and on ragged N.
 */
CORR_API corr_status corr_set_tile(corr_handle h, int32_t tile);

/*
 * Autotuner: time the X-engine with each block size on the first n_spectra
 * held spectra (on max(256, enough channels for four 128-input blocks per
 * workgroup slot of the GPU) channels, at most all, into scratch
 * accumulators, so the integration is untouched), keep the fastest for
 * this handle (the built-in choice unless another is at least 2% faster)
 * and write it
 * to *tile (may be NULL).  Results are cached per (device architecture,
 * precision, inputs rounded up to 64, channels, time blocks, spectra order)
 * for the process, and in the text file named by the environment variable
 * CORR_TUNE_CACHE when it is set.  Synchronises the stream; CORR_E_STATE
 * while the stream is being captured into a graph.
 */
CORR_API corr_status corr_autotune(corr_handle h, int32_t n_spectra, int32_t *tile);

/*
 * Order of the held spectra in device memory: time-block-major (1), channel-
 * major (0) or the built-in rule (-1: time-block-major from 512 inputs or
 * 2048 channels, or when a channel's row of one time block is under 1 KB).
 * Results do not depend on it; speed does.  Changing it drops the held
 * spectra (the next X-engine call needs a new F-engine call).  Batch
 * sub-arrays: CORR_E_STATE.
 */
CORR_API corr_status corr_set_spectra_layout(corr_handle h, int32_t time_block_major);

/* A configuration chosen by corr_autotune_fx. */
typedef struct {
    int32_t tile;             /* X-engine block size, 64 or 128 */
    int32_t time_block_major; /* order of the held spectra (corr_set_spectra_layout) */
    int32_t default_tile;     /* the built-in choices the timings compare against */
    int32_t default_time_block_major;
    float ms_default;         /* F + X time of the built-in choice (-1: taken from the cache) */
    float ms_tuned;           /* F + X time of the chosen configuration (-1: from the cache) */
} corr_tuning;

/*
 * F + X autotuner: times the F-engine (every channel) and the X-engine (on
 * the channels corr_autotune uses, into scratch accumulators, scaled up to
 * all channels)
 * on these voltages for both spectra orders and both block sizes, keeps the
 * fastest for the handle (the built-in choice unless another is at least 2%
 * faster), and channelises the voltages once more in the
 * chosen order, so the handle then holds their spectra as after
 * corr_fengine (the accumulators are not touched).  Arguments as for
 * corr_fengine (n_spectra <= n_integrate).  Results are cached per (device
 * architecture, precision, inputs rounded up to 64, channels, time blocks)
 * for the process and in the file named by CORR_TUNE_CACHE when set.
 * Synchronises the stream; CORR_E_STATE while capturing and for batch
 * sub-arrays.  *out (may be NULL) receives the choice and both timings.  The
 * spectra held before the call are dropped (on an error, none are held).
 */
CORR_API corr_status corr_autotune_fx(corr_handle h, const void *d_volts, int64_t ld_samples, int32_t n_spectra,
                                      const float *d_inv_scale, corr_tuning *out);

/*
 * Batched form: many sub-arrays of uneven size (stations, channels,
 * integration) correlated together.  As in the paper's space-division view
 * of the correlation triangle (Section 4), each sub-array's triangle of
 * pairs is cut into blocks; the (sub-array, channel, block) items of all
 * sub-arrays are drained by persistent X-engine launches -- one per block
 * size in use, so at most two -- from eight per-XCD work queues (channels
 * split evenly, largest items first, idle workgroups take work from the
 * other queues).  A sub-array whose blocks alone number at least four per
 * workgroup the GPU holds at its block size fills the GPU by itself and
 * runs as its own ordinary X-engine launch within the same call (measured
 * faster than the persistent launch for such sub-arrays, whose unbroken
 * load runs at a lower clock).  All sub-arrays share one precision and stream (and one
 * F-engine scratch, since their F-engines run in stream order).  Each
 * sub-array is an ordinary handle owned by the batch (corr_batch_get): use
 * corr_fengine, corr_dump_visibilities and corr_autotune on it as usual;
 * corr_destroy on it is CORR_E_STATE.  Whether a sub-array's accumulators
 * are logically zero is a flag in device memory: set at creation and by a
 * dump with reset, cleared by the next X-engine call on the sub-array, whose
 * items then write their sums instead of adding them (the accumulators are
 * never cleared in memory, and the first call of an integration does not
 * read them).  The flag is written by kernels, not memsets, so a sequence of
 * corr_fengine / corr_xengine_batched calls (with dumps between them, if
 * wanted) can be captured into a HIP graph once a first corr_xengine_batched
 * call with the same n_spectra has been made outside the capture.  A changed work list
 * during capture is CORR_E_STATE; after it changes outside a capture,
 * capture again (an older graph then reads the new work plan, which stays
 * within every sub-array's buffers, but launches only the block sizes it
 * was captured with).
 */
typedef struct corr_batch *corr_batch_handle;

CORR_API corr_status corr_create_batched(const corr_params *params, int32_t n, void *hip_stream,
                                         corr_batch_handle *out);
CORR_API corr_status corr_batch_get(corr_batch_handle b, int32_t i, corr_handle *h);

/* n_spectra: host array [n]; sub-array i correlates its first n_spectra[i]
 * held spectra (0 = skip).  Same checks as corr_xengine per sub-array. */
CORR_API corr_status corr_xengine_batched(corr_batch_handle b, const int32_t *n_spectra);
CORR_API corr_status corr_destroy_batched(corr_batch_handle b);

/*
 * X-engine on caller spectra with no allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The same result as a handle of
 * these params (CORR_TRI_LOWER / CORR_CHAN_MAJOR only) doing
 * corr_xengine(h, d_spectra, n_spectra, d_inv_scale) on zeroed accumulators
 * (accumulate = 0) or on accumulators holding d_vis (accumulate = 1), then
 * a dump to d_vis: no handle, nothing allocated or freed.  Staging lives in a
 * 32 MiB device array of the library, one per device, that every call on the
 * device shares: calls that overlap on one device (other streams or host
 * threads) race and must be serialised by the caller.
 *   params      : n_stations, n_pols, n_channels, precision, layout, order as
 *                 for corr_create (n_integrate and device_mem_cap unused).
 *   d_spectra   : [n_spectra][n_channels][n_inputs][2] public spectra, as
 *                 for corr_xengine (int8: -128 is read as -127), 16-byte
 *                 aligned.
 *   d_inv_scale : FP16 / FP8: the float32 per-channel inv_s[k] (NULL = 1.0);
 *                 NULL for FP32 and int8.
 *   d_vis       : corr_visibility_bytes(params) bytes, 8-byte aligned;
 *                 written (accumulate = 0) or added to (1), in the dump's
 *                 units (int8: raw int32 sums; for int8 the caller keeps the
 *                 total spectra summed into d_vis within
 *                 CORR_INT8_MAX_INTEGRATE).
 *   hip_stream  : the stream the work is enqueued on (asynchronous).
 * Errors: as corr_create for params; CORR_E_INVALID_ARG (pointers, flags);
 * CORR_E_OVERFLOW (int8 over 66572 spectra in one call); CORR_E_UNSUPPORTED
 * when one channel's held spectra (n_inputs x ceil(n_spectra / time block) x
 * 128 bytes, time block as for corr_fengine_at) do not fit the staging array
 * next to the C scales -- about 32 MiB; CORR_E_HIP.
 */
CORR_API corr_status corr_xengine_noalloc(const corr_params *params, const void *d_spectra, int32_t n_spectra,
                                          const float *d_inv_scale, void *d_vis, int32_t accumulate,
                                          void *hip_stream);

/* Static text of a status code. */
CORR_API const char *corr_status_string(corr_status s);

/* Text of the last error recorded on the handle (HIP error strings included);
 * "" if none.  Valid until the next call on the handle. */
CORR_API const char *corr_last_error(corr_handle h);

#ifdef __cplusplus
}
#endif

#endif /* CORR_H */
