// kernels.hpp -- internal launch interface between the C-ABI host code and the
// HIP kernels.  Not part of the public boundary (include/holo.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phase_src.hpp"

namespace holo {

// Launch shapes of one plan (0 = built-in heuristic).  Chosen per
// (path, nx, ny, n_sf) by the autotuner or left at the defaults.
struct LaunchCfg {
    int cols_per_block = 0;        // C of the generation column pass (OSPR K2, GS cols)
    int rows_per_block = 0;        // row transforms per block (OSPR K1, GS rows)
    int ksplit = 0;                // sub-frame groups per reconstruction-row block
    int recon_cols_per_block = 0;  // C of the reconstruction column pass
    int pad = -1;                  // extra elements per row of internal fields (-1 = heuristic)
    int chunk = 0;                 // OSPR sub-frames per generation chunk (0 = all at once)
    int pts = 0;                   // points per thread: GS passes 4, 8 or 16; OSPR K1-K3 8 or 16 (FP32; 0 = per-pass heuristic)
    int prec = 0;                  // DFT stages: 0 FP32 registers, 1 BF16 MFMA, 2 FP16 MFMA (sizes >= 256)
    const void* dftop = nullptr;   // DFT-matrix operand table of `prec` (launch_dft_operand_gen)
};

// Grouped binary OSPR frames: frames of one size and launch shape run each of
// K1..K4 as one launch, blockIdx.y selecting the frame (its table entry) and
// blocks past the frame's own count returning at once.  Every frame keeps the
// shapes (and so the arithmetic) of its single-frame launch; all its
// sub-frames are generated at once (no chunking).
struct GroupFrame {
    const float* target;
    float2* x1;            // n_sf half planes
    uint32_t* bits;        // n_sf * nx * ny / 32 words
    float2* x2;            // n_sf half spectra
    float* recon;          // nx * ny, or null
    double* part;          // 5 per spectrum row
    double* nm;            // {NMSE, NMSE_sym}
    uint64_t c0;           // pool offset of the frame (reduced)
    float inv_scale;       // 1 / (n_sf * nx * ny)
    int n_sf;
    int spb;               // K1: sub-frames per block
    int k1_blocks;         // K1 blocks of the frame
    int k2_tiles;          // K2 column tiles of the frame
};

// Row pitch (complex elements) of the library's internal [rows][nx] fields:
// power-of-two row strides make column passes hit few memory channels, so a
// small pad is added (planned, or 16 elements for nx >= 256).
inline int row_pitch(int nx, const LaunchCfg& c)
{
    const int pad = c.pad >= 0 ? c.pad : (nx >= 256 ? 16 : 0);
    return nx + pad;
}

// Column-tile width for a column pass of length n over ncols columns and
// nbatch independent fields (see the definition for the rule).
int col_block_cols(int n, int ncols, int nbatch, int planned, int cmin);

// FP64 twiddle generation on the device: tw[k] = fp32(exp(-2*pi*i*k/n)).
hipError_t launch_twiddle_gen(float2* tw, int n, hipStream_t s);

// DFT-matrix operand table of the matrix-core radix-16 DFTs (kDftOpElems
// 16-bit values, 8 KiB): prec 1 (BF16) or 2 (FP16), FP64 evaluation on the
// device.
constexpr int kDftOpElems = 2 * 4 * 64 * 8;
hipError_t launch_dft_operand_gen(uint16_t* out, int prec, hipStream_t s);

// Plain unitary 2D transform (Eq. (1) for sign < 0, Eq. (2) for sign > 0):
// rows of `in` into `tmp`, columns of `tmp` into `out` (1/sqrt(N) applied).
hipError_t launch_fft2(const float2* in, float2* tmp, float2* out, int nx, int ny, int sign,
                       const float2* tw_x, const float2* tw_y, const LaunchCfg& cfg, hipStream_t s);

// OSPR K1: R = T * pool phasor, inverse row transform, all n_sf sub-frames.
// The pool position of the launch's first pixel is c0 + *c0_base, reduced mod
// the pool length for the cyclic sources (c0_base may be NULL; both terms
// already reduced).  For SRC_MSEQ, src.rows holds the launch's n_sf*ny row
// states (launch_mseq_rows with the same c0, c0_base).
hipError_t launch_ospr_rows(const float* target, int nx, int ny, int n_sf, const PhaseSrc& src, uint64_t c0,
                            const uint64_t* c0_base, float2* x1, const float2* tw_x, const LaunchCfg& cfg,
                            hipStream_t s);

// OSPR K1 for binary frames: the Hermitian part of R (whose
// inverse transform is Re H), inverse row transform of rows 0..ny/2 only,
// written as half planes of ny/2 + 1 rows (stride (ny/2 + 1) * pitch).
// gtab (device memory): a grouped launch of `ngroup` frames whose grid row
// holds `grid_x` blocks (the largest frame's count); the per-frame arguments
// above are then taken from the table.
hipError_t launch_ospr_rows_h(const float* target, int nx, int ny, int n_sf, const PhaseSrc& src, uint64_t c0,
                              const uint64_t* c0_base, float2* x1, const float2* tw_x, const LaunchCfg& cfg,
                              hipStream_t s, const GroupFrame* gtab = nullptr, int ngroup = 1, int grid_x = 0);

// M-sequence source: Galois state of the first pixel of every (sub-frame,
// row) of a launch, rows[k*ny + y]; aux = x^(2^j) for j < 31, then S_0.
hipError_t launch_mseq_rows(const uint32_t* aux, uint64_t c0, const uint64_t* c0_base, int nx, int ny, int n_sf,
                            uint32_t* rows, hipStream_t s);
// Phasors of pixels (k, y, x) of n_sf sub-frames from pool position c0, as the
// generation kernels draw them: out[(k*ny + y)*nx + x].
hipError_t launch_phase_mask(const PhaseSrc& src, uint64_t c0, int nx, int ny, int n_sf, float2* out,
                             hipStream_t s);
// OSPR K2: inverse column transform, binarise + pack, forward column transform
// of the +-1 column, half spectrum (rows 0..ny/2) out; x1 holds the half
// planes of launch_ospr_rows_h.
hipError_t launch_ospr_cols(const float2* x1, int nx, int ny, int n_sf, uint32_t* bits, float2* x2,
                            const float2* tw_y, const LaunchCfg& cfg, hipStream_t s, const GroupFrame* gtab = nullptr,
                            int ngroup = 1, int grid_x = 0);
// K2 variants: mode OSPR_PAIRS writes sub-frames 2j (Re H) and 2j+1 (Im H) of
// each of the n_fields fields (bits, half spectra); mode OSPR_LEVELS8 writes
// 8-level codes (uint8 [n_fields][ny*nx]) and full column spectra.
enum OsprMode { OSPR_BINARY = 0, OSPR_PAIRS = 1, OSPR_LEVELS8 = 2 };
hipError_t launch_ospr_cols_mode(int mode, const float2* x1, int nx, int ny, int n_fields, void* holo, float2* x2,
                                 const float2* tw_y, const LaunchCfg& cfg, hipStream_t s);
// Reconstruction column transform straight from a quantised hologram:
// levels 2 (packed bits -> half spectrum) or 8 (codes -> full spectrum).
hipError_t launch_recon_cols(const void* holo, int levels, int nx, int ny, int n_sf, float2* x2,
                             const float2* tw_y, const LaunchCfg& cfg, hipStream_t s);
// K3: row transform, |.|^2, mean over sub-frames, NMSE partial sums (FP64).
// half: x2 holds rows 0..ny/2 of a Hermitian-symmetric spectrum.
hipError_t launch_recon_rows(const float2* x2, int nx, int ny, int n_sf, bool half, const float* target,
                             float* recon, double* partials, const float2* tw_x, const LaunchCfg& cfg,
                             hipStream_t s, const GroupFrame* gtab = nullptr, int ngroup = 1);
// K4: deterministic reduction of `nrows` x 5 partials -> {NMSE, NMSE_sym}.
hipError_t launch_nmse_finalize(const double* partials, int nrows, double* out2, hipStream_t s);

// Single-frame launch shapes, for building a group: K1 blocks and sub-frames
// per block; K2 tiles; K3 sub-frame groups per block.
void ospr_rows_h_shape(int nx, int ny, int n_sf, const LaunchCfg& cfg, int* blocks, int* spb);
int ospr_cols_tiles(int nx, int ny, int n_sf, const LaunchCfg& cfg);
int recon_rows_groups(int nx, int n_sf, const LaunchCfg& cfg);
// K1..K4 of the `n` frames of table `tab` (device memory; the host copy
// `host` gives the grid), all of size nx x ny with launch shapes `cfg`.
hipError_t launch_ospr_group(const GroupFrame* tab, const GroupFrame* host, int n, int nx, int ny,
                             const PhaseSrc& src, const uint64_t* c0_base, const float2* tw_x, const float2* tw_y,
                             const LaunchCfg& cfg, hipStream_t s);

// Gerchberg-Saxton passes.
enum GsRowMode { GS_INIT = 0, GS_ITER = 1, GS_FINAL = 2 };
struct GsConsts {
    double sum_t2, sum_t4, te_scale;
};
// One frame of a grouped GS launch (frames of one size iterate together,
// blockIdx.y -- blockIdx.x for the one-block-per-frame kernels -- selecting
// the frame); the per-frame arguments of the launchers below come from here.
struct GsFrame {
    const float* target;
    const float2* init;    // caller seed phasors, or null (pool seed)
    float2* state;         // [ny][pitch] working field
    float2* field;         // unitary replay field out [ny][nx]
    uint8_t* codes;        // 8-level codes out, or null
    double* pinit;         // [ny][2] INIT partials
    double* piter;         // [n_iter][ny][3] iteration partials
    GsConsts* consts;
    double* nmse;          // [n_iter], or null
    double* err;           // [n_iter], or null
    uint64_t c0;           // pool offset of the frame (reduced)
};
// GS_INIT reads the pool at c0 + *c0_base (c0_base may be NULL).  gtab: a
// grouped launch of `ngroup` frames; `part_off` then offsets the frame's
// partials (iteration it: it * 3 * ny).
hipError_t launch_gs_rows(int mode, const float* target, int nx, int ny, const PhaseSrc& src, uint64_t c0,
                          const uint64_t* c0_base, const float2* init, float2* state, float2* field_out,
                          double* partials, const GsConsts* consts, const float2* tw_x,
                          const LaunchCfg& cfg, hipStream_t s, const GsFrame* gtab = nullptr, int ngroup = 1,
                          int part_off = 0);
// gtab: grouped launch; with it, codes != null asks for every frame's codes.
hipError_t launch_gs_cols(float2* state, int nx, int ny, uint8_t* codes, const float2* tw_y,
                          const LaunchCfg& cfg, hipStream_t s, const GsFrame* gtab = nullptr, int ngroup = 1);
hipError_t launch_gs_consts(const double* init_partials, int ny, int nx, GsConsts* consts, hipStream_t s,
                            const GsFrame* gtab = nullptr, int ngroup = 1);
hipError_t launch_gs_finalize(const double* partials, int n_iter, int ny, const GsConsts* consts,
                              double* nmse_out, double* err_out, hipStream_t s, const GsFrame* gtab = nullptr,
                              int ngroup = 1);

}  // namespace holo
