/*
 * holo.h -- C ABI of the MI355X (gfx950) hot path for LUT-based phase
 * randomisation in hologram generation, after Christopher & Wilkinson,
 * "Lookup tables for phase randomisation in hardware generated holograms"
 * (arXiv:2004.04049).
 *
 * The paper poses hologram generation as finding the aperture f whose
 * far-field DFT (Eq. (1)) matches a target; algorithms back-propagate the
 * target with Eq. (2), quantise each pixel to the nearest value the SLM
 * allows, and judge the replay R' = F{H'} (Section 2).  Targets are amplitudes
 * only, so a random phase is attached to them (Section 3), drawn here from a
 * small table read cyclically (Sections 4 and 5) instead of a PRNG plus
 * sin/cos.
 *
 * Conventions for every call:
 *   - Images are row-major [ny][nx] (x fastest), raster index p = y*nx + x.
 *   - "device" buffers live in the GPU's memory and are owned by the caller
 *     (e.g. torch tensors passed by data_ptr()); the library never frees them.
 *     "host" buffers are ordinary process memory.
 *   - Complex fields are interleaved float pairs (re, im), 8 bytes per pixel.
 *   - nx and ny must be powers of two in [16, 2048] (HOLO_EUNSUPPORTED
 *     otherwise).
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Device
 *     outputs are written in stream order; the call returns after enqueueing,
 *     except that host outputs (NMSE values) are complete on return, which
 *     synchronises the stream.  With HOLO_F_NMSE_DEVICE the NMSE pointers are
 *     device pointers written in stream order and nothing synchronises.
 *   - Calls made concurrently on different host threads are safe; calls that
 *     overlap on the same stream are ordered by it.  The library keeps one
 *     scratch workspace per (device, stream).  While one call captures a new
 *     HIP graph (graph replay on, the first call of a shape), the library's
 *     other calls wait: the HIP runtime can invalidate a capture when another
 *     thread launches or allocates meanwhile.  GPU work that the caller
 *     enqueues from other threads through other libraries during such a
 *     capture is not covered; a call whose capture was invalidated returns
 *     HOLO_EDEVICE (holo_set_graphs(0) avoids captures altogether).
 *   - Every call returns a holo_status; no exception or abort crosses the ABI.
 *     holo_last_error() gives this thread's text for the last failure.
 *   - Environment switches, read at each use (so they may change between
 *     calls), to exercise the failure paths:
 *       HOLO_WORKSPACE_CAP=<bytes>  a call whose scratch workspace would
 *                                   exceed the cap returns HOLO_ENOMEM;
 *       HOLO_DEBUG_FAIL=device      every kernel or graph launch returns
 *                                   HOLO_EDEVICE before it is enqueued;
 *       HOLO_DEBUG_POISON=1         each call's workspace is filled with
 *                                   0xFF bytes (NaN) before its kernels run.
 */
#ifndef HOLO_H_
#define HOLO_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOLO_API __attribute__((visibility("default")))

typedef int32_t holo_status;
enum {
    HOLO_OK = 0,
    HOLO_EINVAL = -1,       /* null required pointer or out-of-range count   */
    HOLO_EUNSUPPORTED = -2, /* size or precision the library does not handle */
    HOLO_ENOMEM = -3,       /* workspace or table allocation failed          */
    HOLO_EDEVICE = -4       /* a HIP call failed; text in holo_last_error()  */
};

/* Arithmetic of the transform stages.
 *   HOLO_FP32  radix stages in FP32 on the vector ALUs.
 *   HOLO_BF16, HOLO_FP16  the 16-point DFTs of every radix-16 stage of
 *              every transform as DFT-matrix products on the matrix cores:
 *              data rounded once per radix-16 stage to BF16 (8 significant
 *              bits) or FP16 (11), DFT matrix split into two operand-format
 *              terms (hi + lo), FP32 accumulation; inter-stage twiddles, the
 *              last radix-2/4/8 stage, pointwise steps and all sums stay
 *              FP32/FP64.  Sides of 256 and more only.  Results are
 *              not bit-exact: binarisation flips pixels whose Re H is within
 *              the rounding error of 0.
 * Entry points that take a precision return HOLO_EUNSUPPORTED for BF16/FP16
 * below 256 and HOLO_EINVAL for other values. */
enum { HOLO_FP32 = 0, HOLO_BF16 = 1, HOLO_FP16 = 2 };

/* Flags.  HOLO_F_OSPR_PAIRS and HOLO_F_OSPR_LEVELS8 select an OSPR variant
 * (holo_ospr_generate, holo_ospr_generate_batched); neither is the paper's
 * method, which is the default binary frame. */
enum { HOLO_F_NMSE_DEVICE = 1, HOLO_F_OSPR_PAIRS = 2, HOLO_F_OSPR_LEVELS8 = 4 };

/* holo_lut_check() warning bits (Section 5.1 hard limits, Section 8 rules). */
enum {
    HOLO_LUT_FLAT = 1,           /* n_lut == 0: no randomisation at all          */
    HOLO_LUT_NOT_PRIME = 2,      /* length not prime (Section 8, first rule)     */
    HOLO_LUT_LE_NSF = 4,         /* n_lut <= n_sf: sub-frames not independent   */
    HOLO_LUT_LE_MAXDIM = 8,      /* n_lut <= max(nx, ny) (Section 8, third rule) */
    HOLO_LUT_DIVIDES_FRAME = 16, /* n_lut divides nx*ny: identical sub-frames    */
    HOLO_LUT_LT_FULL = 32        /* n_lut < nx*ny*n_sf: not PRNG-equivalent     */
};

typedef struct holo_lut holo_lut; /* opaque, library-owned, immutable once built */

HOLO_API const char* holo_last_error(void);
HOLO_API int32_t holo_version(void);

/* ---------------------------------------------------------------------------
 * Phase LUT (Section 4: a pool of random phases fixed ahead of time).
 *
 * Every entry point that draws random phases takes a holo_lut handle and reads
 * its pool at positions c + k*nx*ny + p (Section 5, Fig. 3); the handle decides
 * how a position becomes a unit phasor.  Handles are immutable and live on the
 * device current at creation; holo_lut_free releases any of them.
 *
 * holo_lut_build (HOLO_SRC_TABLE, the method as published): n_lut phases
 * phi_j = 2*pi*u_j, u_j = (x_j >> 11) * 2^-53 from SplitMix64 seeded with
 * `seed` (x_j = output j; uniform on [0, 2*pi)); the device holds them as FP32
 * unit phasors (cos phi_j, sin phi_j) so no trigonometry runs per pixel.
 * n_lut = 0 builds the flat-phase table (phasor 1).  n_lut must be < 2^29
 * (HOLO_EUNSUPPORTED): the kernels address the table with 32-bit byte offsets.
 * holo_lut_from_phases: the same from caller phases (host, FP64, n_lut).
 *
 * holo_lut_build_codes (HOLO_SRC_CODES8; the one-byte-per-entry reading of the
 * LUT storage figure of Section 5.2): n_lut 8-bit codes q_j = x_j >> 56 of the
 * same SplitMix64 outputs, phase 2*pi*q_j/256; the device holds one byte per
 * entry and the 256 phasors exp(2*pi*i*q/256) (FP64, rounded to FP32).
 * 1 <= n_lut < 2^31.
 *
 * holo_lut_prng (HOLO_SRC_PRNG; Section 4's software route, a PRNG plus
 * trigonometric functions): no table.  Position i (unbounded, the cursor taken
 * mod 2^64) gets x_i = SplitMix64 output i of `seed` in counter form (the x_j
 * of holo_lut_build, so the pool is an endless table of that seed), phase
 * 2*pi*floor(2^24 * u_i)/2^24 (u_i as above, truncated to 24 bits), phasor from
 * the GPU's FP32 sine/cosine evaluated on the device at each use.
 *
 * holo_lut_mseq (HOLO_SRC_MSEQ; Section 7's M-sequence alternative, which
 * still needs sine and cosine tables): bits s_n of the binary M-sequence of the
 * primitive trinomial x^31 + x^3 + 1, s_{n+31} = s_{n+3} xor s_n, with s_0..s_30
 * = bits 30..0 of (SplitMix64 output 0 of `seed`) & (2^31 - 1) (1 if that is 0);
 * position i gets code q_i = bits s_{8i}..s_{8i+7} (s_{8i} most significant),
 * phase 2*pi*q_i/256, phasor from the 256-entry table.  Period 2^31 - 1, so it
 * behaves as a pool of n_lut = 2^31 - 1 entries.
 *
 * holo_lut_kind: HOLO_SRC_* of a handle (-1 for NULL).
 * holo_lut_size: n_lut (PRNG: UINT64_MAX; MSEQ: 2^31 - 1).
 * holo_lut_phases: copies min(n, n_lut) FP64 phases to host `out` (TABLE,
 * CODES8); HOLO_EUNSUPPORTED for PRNG and MSEQ, which keep no table.
 * holo_lut_check: bitmask of HOLO_LUT_* warnings; never an error, because the
 * paper's own sweeps break these rules on purpose.
 * ------------------------------------------------------------------------- */
enum { HOLO_SRC_TABLE = 0, HOLO_SRC_CODES8 = 1, HOLO_SRC_PRNG = 2, HOLO_SRC_MSEQ = 3 };
HOLO_API holo_status holo_lut_build(uint64_t n_lut, uint64_t seed, holo_lut** out);
HOLO_API holo_status holo_lut_from_phases(const double* phases, uint64_t n_lut, holo_lut** out);
HOLO_API holo_status holo_lut_build_codes(uint64_t n_lut, uint64_t seed, holo_lut** out);
HOLO_API holo_status holo_lut_prng(uint64_t seed, holo_lut** out);
HOLO_API holo_status holo_lut_mseq(uint64_t seed, holo_lut** out);
HOLO_API int32_t holo_lut_kind(const holo_lut* lut);
HOLO_API holo_status holo_lut_phases(const holo_lut* lut, double* out, uint64_t n);
HOLO_API uint64_t holo_lut_size(const holo_lut* lut);
HOLO_API void holo_lut_free(holo_lut* lut);
HOLO_API uint32_t holo_lut_check(uint64_t n_lut, int64_t nx, int64_t ny, int32_t n_sf);

/* ---------------------------------------------------------------------------
 * holo_ospr_generate -- One-Step Phase-Retrieval frame (Section 2, 3).
 *
 * For sub-frames k = 0..n_sf-1: R_k = T * exp(i*phi), with phi read from the
 * LUT at (c + k*nx*ny + p) mod n_lut, c = *cursor (Section 5, Fig. 3);
 * H_k = F^{-1}{R_k} (Eq. (2)); each pixel set to the nearest of {+1, -1}, i.e.
 * bit = (Re H_k < 0), tie Re H = 0 -> +1 (bit 0); replay I_k = |F{H'_k}|^2
 * (Eq. (1), unitary); time average I = (1/n_sf) sum_k I_k (Section 3).
 *   target     device float[ny][nx], amplitudes (any non-negative scale)
 *   cursor     host in/out; advanced by n_sf*nx*ny on success (pair mode:
 *              n_sf/2*nx*ny)
 *   holo_out   device uint32[n_sf][nx*ny/32] packed bits: bit p%32 of word
 *              p/32 is pixel p (LSB first); 1 means phase pi.  With
 *              HOLO_F_OSPR_LEVELS8: uint8 codes [n_sf][ny][nx] instead.
 *   recon      device float[ny][nx] time-averaged intensity, or NULL
 *   nmse2      {NMSE vs T^2, NMSE vs the point-symmetrised T^2} or NULL, where
 *              NMSE(I, W) = 1 - (sum I W)^2 / (sum I^2 * sum W^2), the
 *              optimal-scale normalised MSE, accumulated in FP64
 *   precision  HOLO_FP32, HOLO_BF16 or HOLO_FP16 (stages of all transforms)
 *   flags      HOLO_F_NMSE_DEVICE, and at most one variant (not the paper's):
 *     HOLO_F_OSPR_PAIRS: each randomised field H_j, j < n_sf/2 (pool index
 *       k = j above), gives two binary sub-frames, 2j from Re H_j and 2j+1
 *       from Im H_j (bit = part < 0); n_sf must be even.  Half the inverse
 *       transforms and pool draws of the binary frame.
 *     HOLO_F_OSPR_LEVELS8: sub-frame k is quantised to the nearest of the
 *       eight phases exp(i*2*pi*m/8), m = round(8 arg H_k/(2 pi)) mod 8,
 *       H = 0 -> 0, and replayed as such.
 * Errors: HOLO_EINVAL for null target/lut/cursor/holo_out, n_sf < 1, both
 * variant flags, or an odd n_sf in pair mode.
 * ------------------------------------------------------------------------- */
HOLO_API holo_status holo_ospr_generate(const float* target, int64_t nx, int64_t ny, int32_t n_sf,
                                        const holo_lut* lut, uint64_t* cursor, void* holo_out,
                                        float* recon, double* nmse2, int32_t precision, uint32_t flags,
                                        void* hip_stream);

/* ---------------------------------------------------------------------------
 * holo_gs_iterate -- Gerchberg-Saxton (Section 2), phase-only hologram,
 * amplitude-only replay constraint.
 *   R_0 = T * phasor, phasor = init_phasor/|init_phasor| (0 -> 1) if given,
 *         else the LUT at (c + p) mod n_lut, c = *cursor (then *cursor += N);
 *   iteration i = 1..n_iter: H_i = F^{-1}{R_{i-1}}, H'_i = H_i/|H_i|
 *         (0 -> 1), R'_i = F{H'_i}, NMSE_i = NMSE(|R'_i|^2, T^2),
 *         E_i = sum (|R'_i| - Te)^2 with Te = T*sqrt(N/sum T^2),
 *         R_i = T * R'_i/|R'_i| (0 -> T);
 *   then the final H_n is quantised to 8 levels m = round(8 arg H/(2 pi)) mod 8
 *   and its replay is reconstructed.
 *   target       device float[ny][nx]
 *   init_phasor  device float2[ny][nx] or NULL (LUT).  Passing a previous
 *                call's `field` resumes the iteration exactly.
 *   field        device float2[ny][nx] out: unitary replay field R'_n, or NULL
 *   codes        device uint8[ny][nx] out: 8-level codes of H_n, or NULL
 *   nmse_per_iter, err_per_iter   [n_iter] or NULL (host, or device with
 *                HOLO_F_NMSE_DEVICE)
 *   nmse_final2  NMSE pair of the 8-level replay, or NULL (needs codes)
 *   recon        device float[ny][nx] 8-level replay intensity, or NULL
 * Errors: HOLO_EINVAL for null target/cursor, null lut without init_phasor,
 * n_iter < 1, nmse_final2/recon without codes.
 * ------------------------------------------------------------------------- */
HOLO_API holo_status holo_gs_iterate(const float* target, int64_t nx, int64_t ny, int32_t n_iter,
                                     const holo_lut* lut, uint64_t* cursor, const float* init_phasor,
                                     float* field, uint8_t* codes, double* nmse_per_iter, double* err_per_iter,
                                     double* nmse_final2, float* recon, int32_t precision, uint32_t flags,
                                     void* hip_stream);

/* ---------------------------------------------------------------------------
 * holo_gs_iterate_batched -- holo_gs_iterate (Section 2) on n_frames frames of
 * one size at once, each exactly as a holo_gs_iterate call computes it, with
 * the pool cursor continuing from frame to frame in array order: a
 * pool-seeded frame starts at *cursor + N * (pool-seeded frames before it),
 * and *cursor advances by N per pool-seeded frame.  Every pass of every
 * iteration is one launch over all frames (blockIdx.y selects the frame):
 * GS iterations of one frame are sequential, and one 512^2 or 1024^2 frame
 * leaves most of the GPU waiting on the dependent stages of its passes;
 * independent frames fill it.
 *   frames         host array of n_frames (1..256) descriptors; device
 *                  pointers as holo_gs_iterate's: target, init_phasor (NULL:
 *                  pool seed), field, codes, recon (each may be NULL except
 *                  target; recon needs the frame's codes)
 *   nmse_per_iter, err_per_iter  [n_frames][n_iter] or NULL
 *   nmse_final2    [n_frames][2] or NULL (needs codes on every frame)
 *                  (host, or device with HOLO_F_NMSE_DEVICE)
 * The work is captured into a HIP graph and replayed while frames, buffers
 * and plan are unchanged (launched directly on the legacy default stream or
 * while kernel timing is on).  FP32 only.
 * Errors: HOLO_EINVAL (null frames/cursor/target, n_frames or n_iter out of
 * range, recon or nmse_final2 without codes, null lut with a pool-seeded
 * frame), HOLO_EUNSUPPORTED (sizes; the M-sequence source, whose per-row
 * states this call does not prepare).
 * ------------------------------------------------------------------------- */
typedef struct {
    const float* target;       /* device float[ny][nx]                   */
    const float* init_phasor;  /* device float2[ny][nx], or NULL (pool)  */
    float* field;              /* device float2[ny][nx] out, or NULL     */
    uint8_t* codes;            /* device uint8[ny][nx] out, or NULL      */
    float* recon;              /* device float[ny][nx] out, or NULL      */
} holo_gs_frame;

HOLO_API holo_status holo_gs_iterate_batched(const holo_gs_frame* frames, int32_t n_frames, int64_t nx, int64_t ny,
                                             int32_t n_iter, const holo_lut* lut, uint64_t* cursor,
                                             double* nmse_per_iter, double* err_per_iter, double* nmse_final2,
                                             uint32_t flags, void* hip_stream);

/* ---------------------------------------------------------------------------
 * holo_gs_iterate_noalloc -- holo_gs_iterate for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, computation and results as
 * holo_gs_iterate (the same kernels and launch plan), except:
 *   - The call's scratch (the iterated field, per-iteration partial sums,
 *     the replay spectrum, the NMSE values) is a fixed device buffer of
 *     HOLO_GS_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held
 *     until the process ends; no call allocates or frees anything and no
 *     graph is captured.  A problem whose scratch would exceed the buffer
 *     returns HOLO_EUNSUPPORTED before anything is enqueued (1024^2 with codes
 *     and a caller field fits about 570 iterations; 2048^2 does not fit).
 *   - nmse_per_iter, err_per_iter and nmse_final2 are device pointers and
 *     flags must include HOLO_F_NMSE_DEVICE when any of them is given
 *     (HOLO_EINVAL otherwise); the call never synchronises its stream, except
 *     that the first call on a device generates the fixed twiddle tables and
 *     waits for them (HOLO_EUNSUPPORTED if that first call is made under
 *     stream capture).
 *   - Every call on one GPU shares that GPU's buffer, which keeps the last
 *     call's contents (everything a call reads it first writes): calls that
 *     overlap on one GPU, on different streams or unordered host threads,
 *     race and must be ordered by the caller.
 *   - Kernel timing (holo_prof_enable) is not recorded for this call.
 * ------------------------------------------------------------------------- */
#define HOLO_GS_NOALLOC_SCRATCH_BYTES (32u << 20)
HOLO_API holo_status holo_gs_iterate_noalloc(const float* target, int64_t nx, int64_t ny, int32_t n_iter,
                                             const holo_lut* lut, uint64_t* cursor, const float* init_phasor,
                                             float* field, uint8_t* codes, double* nmse_per_iter,
                                             double* err_per_iter, double* nmse_final2, float* recon,
                                             int32_t precision, uint32_t flags, void* hip_stream);

/* ---------------------------------------------------------------------------
 * holo_reconstruct_nmse -- replay of quantised holograms, R' = F{H'}
 * (Section 2), intensity time-averaged over n_sf holograms (Section 3).
 *   holo    device: levels == 2 -> packed bits as holo_ospr_generate writes
 *           them, [n_sf][nx*ny/32]; levels == 8 -> uint8 codes [n_sf][ny][nx]
 *           meaning exp(i*2*pi*m/8)
 *   recon   device float[ny][nx] or NULL;  nmse2 as in holo_ospr_generate
 * Errors: HOLO_EINVAL for null holo/target, levels not 2 or 8, n_sf < 1.
 * ------------------------------------------------------------------------- */
HOLO_API holo_status holo_reconstruct_nmse(const void* holo, int32_t levels, int64_t nx, int64_t ny,
                                           int32_t n_sf, const float* target, float* recon, double* nmse2,
                                           uint32_t flags, void* hip_stream);

/* ---------------------------------------------------------------------------
 * holo_ospr_generate_batched -- many OSPR frames of uneven size in one call,
 * each exactly as holo_ospr_generate would compute it with the pool cursor
 * continuing from frame to frame in array order (Section 5: frames continue
 * where the previous left off): frame f starts at *cursor + sum over g < f of
 * n_sf_g * nx_g * ny_g, and *cursor advances by the total.  The variant flags
 * of holo_ospr_generate apply to every frame (pair mode: n_sf_g/2 fields each;
 * holo_bits then holds codes for HOLO_F_OSPR_LEVELS8).
 *   frames    host array of n_frames (1..4096) descriptors; every pointer in
 *             them is a device pointer owned by the caller
 *   nmse_out  [n_frames][2] {NMSE, NMSE_sym} per frame, host (complete on
 *             return) or device with HOLO_F_NMSE_DEVICE, or NULL
 * The device work of a batch is captured once into a HIP graph and replayed
 * with one graph launch per call while the frame list, plans and buffers are
 * unchanged; the moving cursor is read from device memory, so replays need
 * no re-capture.  In the graph, binary frames drawn from the table, code or
 * PRNG sources are grouped: frames of one size and launch plan run each pass
 * (row pass, column pass, reconstruction, NMSE) as one launch over up to
 * 64 MiB of half planes, every frame with planes of its own within its
 * unit, the units of a branch reusing one region (plus a frame table that
 * lives with the graph); other frames run their own launches.  Units run on four concurrent branches, longest first.  Results
 * equal the single-frame calls bit for bit either way.  On the legacy default
 * stream, or while kernel timing is on, the frames are launched one by one
 * directly instead.
 * Errors: HOLO_EINVAL (null frames/cursor/target/bits, n_sf < 1, n_frames out
 * of range), HOLO_EUNSUPPORTED (sizes, precision not built).
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t nx, ny;
    int32_t n_sf;
    const float* target;  /* device float[ny][nx]                        */
    void* holo_bits;      /* device: bits uint32[n_sf][nx*ny/32] or codes */
                          /* uint8[n_sf][ny][nx], as holo_ospr_generate    */
    float* recon;         /* device float[ny][nx] time average, or NULL  */
} holo_frame;

HOLO_API holo_status holo_ospr_generate_batched(const holo_frame* frames, int32_t n_frames, const holo_lut* lut,
                                                uint64_t* cursor, double* nmse_out, int32_t precision,
                                                uint32_t flags, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Learned GS seed (not part of the paper's method: a learned replacement for
 * the LUT seed of R_0, trained on the project's own GS output; the LUT seed of
 * holo_gs_iterate remains the fallback).
 * Network: five 3x3 convolutions with circular padding, 1 -> 32 -> 32 -> 32
 * -> 32 -> 2 channels, ReLU after the first four, output phasor o/|o| per
 * pixel.  BF16 weights and activations, FP32 accumulation (the 32->32 layers
 * on MFMA); FP32 master parameters and Adam moments.
 * Parameters: flat FP32 vector of holo_cnn_nparams() values, per layer
 * w[co][ci][3][3] then b[co]; tap (dy, dx) multiplies input (y+dy, x+dx).
 * Loss: L = 1 - |sum w p conj(q)| / sum w, w = T^2, q = label/|label| (any
 * complex label field, e.g. holo_gs_iterate's `field`): the T^2-weighted
 * phase error at the best global phase offset.
 *   holo_cnn_create   He-uniform init from SplitMix64(seed), biases 0
 *   holo_cnn_infer    target device float[ny][nx] -> phasor_out device
 *                     float2[ny][nx] (stream-ordered)
 *   holo_cnn_loss_grad  loss and parameter gradient (host outputs, sync)
 *   holo_cnn_train_step  one Adam (lr) step on a batch: targets device
 *                     float[batch][ny][nx], labels device float2[batch][ny][nx];
 *                     the gradient and loss are the means over the batch
 *                     (per-image forward/backward, gradients accumulated in
 *                     FP32); loss_out host (synchronises) or NULL
 *   holo_cnn_save / holo_cnn_load  parameters, Adam moments and step
 * Images: nx, ny powers of two in [64, 2048].  The network and its scratch
 * live on the device current at creation.
 * ------------------------------------------------------------------------- */
typedef struct holo_cnn holo_cnn;
HOLO_API int32_t holo_cnn_nparams(void);
HOLO_API holo_status holo_cnn_create(uint64_t seed, holo_cnn** out);
HOLO_API holo_status holo_cnn_get_params(const holo_cnn* cnn, float* host_out, int32_t n);
HOLO_API holo_status holo_cnn_set_params(holo_cnn* cnn, const float* host_in, int32_t n);
HOLO_API holo_status holo_cnn_infer(holo_cnn* cnn, const float* target, int64_t nx, int64_t ny, float* phasor_out,
                                    void* hip_stream);
HOLO_API holo_status holo_cnn_loss_grad(holo_cnn* cnn, const float* target, const float* label, int64_t nx,
                                        int64_t ny, double* loss_out, float* grad_out, void* hip_stream);
HOLO_API holo_status holo_cnn_train_step(holo_cnn* cnn, const float* targets, const float* labels, int32_t batch,
                                         int64_t nx, int64_t ny, float lr, double* loss_out, void* hip_stream);
HOLO_API holo_status holo_cnn_save(const holo_cnn* cnn, const char* path);
HOLO_API holo_status holo_cnn_load(const char* path, holo_cnn** out);
HOLO_API void holo_cnn_free(holo_cnn* cnn);

/* ---------------------------------------------------------------------------
 * holo_fft2 -- the unitary transform pair itself: Eq. (1) for sign = -1,
 * Eq. (2) for sign = +1, complex [ny][nx] device in -> device out (may alias),
 * with the stage arithmetic `precision` (HOLO_FP32, HOLO_BF16, HOLO_FP16).
 * ------------------------------------------------------------------------- */
HOLO_API holo_status holo_fft2(const float* in, float* out, int64_t nx, int64_t ny, int32_t sign,
                               int32_t precision, void* hip_stream);

/* ---------------------------------------------------------------------------
 * holo_phase_mask -- the random phasors a generation call would draw (Section
 * 5, Fig. 3): out[(k*ny + y)*nx + x] = phasor of pool position
 * cursor + k*nx*ny + y*nx + x, for k < n_sf, as interleaved (re, im) FP32 pairs
 * in caller-owned device memory of n_sf*ny*nx*8 bytes.  Runs the same device
 * code as the OSPR row pass.  The cursor is not advanced.  nx, ny: powers of two
 * in [16, 2048] (HOLO_EUNSUPPORTED); n_sf >= 1, out and lut non-NULL
 * (HOLO_EINVAL).
 * ------------------------------------------------------------------------- */
HOLO_API holo_status holo_phase_mask(const holo_lut* lut, uint64_t cursor, int64_t nx, int64_t ny, int32_t n_sf,
                                     float* out, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Launch plans and the autotuner (implementation choices, not part of the
 * method: every plan computes the same holograms, except that the points per
 * thread change the FP32 factorisation and so the rounding).
 * A plan is seven ints {cols, rows, ksplit, recon_cols, pad, chunk, pts}:
 * column-tile width of the generation column pass (OSPR: 8 or 16; GS: 2, 4, 8
 * or 16), row transforms per block of the row pass, sub-frame groups per
 * block of the reconstruction row pass, column-tile width of the
 * reconstruction column pass (0 selects the built-in heuristic for these
 * four); extra elements per row of the library's internal fields (-1:
 * heuristic); OSPR sub-frames generated per chunk (0: all; a chunk's
 * intermediate planes are reused, so they can stay in the last-level cache);
 * and points per thread, i.e. the radix factorisation of the transforms: GS
 * passes 4, 8 or 16 (0: heuristic, more threads per transform when a single
 * field offers few transforms; the heuristic and the autotuner use 8 or 16
 * only, as 4 rounds more often); OSPR row, column and reconstruction-row
 * passes all 16 (radix-16 stages, then one radix-2/4/8 stage) or all 8
 * (radix-8 stages, then one radix-2/4 stage), or 0: 8 for the row pass,
 * for column transforms of up to 1024 points and for reconstruction
 * transforms of up to 512, 16 for longer ones (FP32 only: the BF16/FP16 forms take 16;
 * 2048-point columns at 8 points per thread use 8-column tiles).  Plans
 * are keyed by kind (0 = OSPR, 1 = GS), nx, ny and n_sf (ignored for GS); an
 * OSPR plan set with n_sf = 0 serves every sub-frame count of that size that
 * has no plan of its own (holo_plan_get reports the plan a call would use).
 * holo_autotune_ospr / holo_autotune_gs time candidate plans on the caller's
 * inputs (coordinate descent, after a warm-up of the default plan; a
 * candidate's time is the fastest of three batches of `reps` runs;
 * 41 candidates for OSPR, so 20-run batches of a 0.12 ms frame take well under
 * a second) and keep the fastest
 * whose holograms (bits / codes) equal those of the default plan exactly and
 * whose NMSE agrees to 1e-6 relative (FP32 summation order of the average);
 * OSPR candidates with other points per thread than the default (0, 16
 * and 8 are searched jointly with the tile width and chunking) are kept when
 * at most 1e-5 of the bits differ and the NMSE agrees to 1e-6 relative;
 * GS points-per-thread candidates are kept when codes differ on at most 1e-3
 * of the pixels and the per-iteration NMSE agrees to 1e-5 relative after four
 * iterations.  `chosen` (int[7] or NULL) receives the plan.  scratch_bits: device
 * uint32[n_sf][nx*ny/32], overwritten.  holo_plan_save / holo_plan_load
 * write and read all plans as JSON.  holo_set_graphs(0) disables the HIP
 * graph replay of holo_gs_iterate, holo_gs_iterate_batched and
 * holo_ospr_generate_batched (on by default; at most 32 graphs are kept, the
 * oldest destroyed once its own stream has drained).
 * ------------------------------------------------------------------------- */
HOLO_API holo_status holo_autotune_ospr(const float* target, int64_t nx, int64_t ny, int32_t n_sf,
                                        const holo_lut* lut, uint32_t* scratch_bits, int32_t reps, int32_t* chosen,
                                        void* hip_stream);
HOLO_API holo_status holo_autotune_gs(const float* target, int64_t nx, int64_t ny, const holo_lut* lut,
                                      int32_t reps, int32_t* chosen, void* hip_stream);
HOLO_API holo_status holo_plan_set(int32_t kind, int64_t nx, int64_t ny, int32_t n_sf, const int32_t* cfg7);
HOLO_API holo_status holo_plan_get(int32_t kind, int64_t nx, int64_t ny, int32_t n_sf, int32_t* cfg7);
HOLO_API holo_status holo_plan_save(const char* path);
HOLO_API holo_status holo_plan_load(const char* path);
HOLO_API holo_status holo_set_graphs(int32_t on);

/* ---------------------------------------------------------------------------
 * Kernel timing (measurement support, not part of the method).
 * holo_prof_enable(1) makes every subsequent launch record a pair of HIP
 * events on its stream; holo_prof_read waits for the recorded events and
 * returns the accumulated duration (ms) and launch count of one kernel:
 * "ospr_rows", "ospr_cols", "recon_cols", "recon_rows", "nmse_finalize",
 * "gs_rows", "gs_cols", "gs_consts", "gs_finalize", "fft2".  Unknown names
 * read as zero.  holo_prof_reset clears the totals.
 * ------------------------------------------------------------------------- */
HOLO_API holo_status holo_prof_enable(int32_t on);
HOLO_API holo_status holo_prof_read(const char* kernel, double* total_ms, int64_t* count);
HOLO_API void holo_prof_reset(void);

/* Releases every workspace and twiddle table on every device. */
HOLO_API void holo_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* HOLO_H_ */
