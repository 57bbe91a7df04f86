// Internal definitions shared by the HIP kernels and the host runtime of the
// fast template periodogram library (gfx950).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ftp {

constexpr int kMaxH = 11;             // D = 6H - 2 <= 64
constexpr int kTileCells = 2048;      // spreading tile (cells per workgroup)
constexpr int kTileShift = 11;        // log2(kTileCells)
constexpr int kFixedShift = 60;       // fixed-point scale 2^60 for exact accumulation
constexpr int kMaxPasses = 4;
constexpr int64_t kScanSingleMax = 1024 * 16;   // tile counts the one-workgroup scan handles (16 per thread)
constexpr int64_t kLcBlock = 1024;   // pairs per entry of the lightcurve hint table of a batch
constexpr int kTwiddleN = 4096;       // size of the in-LDS twiddle table (w_4096^r)

// Per-lightcurve record.  The host fills the plan part; k_prep_stats fills the
// statistics part on the device.
struct LcInfo {
  int64_t obs_off, n_obs;
  int64_t freq_off, n_f;
  double df;
  int64_t grid_off[2];     // element offset of the w grid (0) and y grid (1)
  int64_t tile_base[2];    // first global tile index of each grid
  int64_t mc[2];           // centre mode of each grid
  double beta[2];          // Gaussian exponent per cell^2 of each grid
  double dec_a[2];         // deconvolution of mode m: dec_a exp(dec_b (m - mc)^2),
  double dec_b[2];         //   dec_a = sqrt(beta / pi), dec_b = pi^2 / (n^2 beta)
  int log2n[2];
  int npass[2];
  int lp[2][kMaxPasses];   // log2 sizes of the FFT passes (largest stride first)
  int msp;                 // kernel half-width in cells
  int stat_nb;             // workgroups of the statistics kernel for this lightcurve
  double yoff;             // fixed offset subtracted from y (shared-phase bands)
  int64_t stat_off;        // slot of its first workgroup's partials
  // filled on the device
  double tref, ybar, yy, inv_sqrt_yy, winv;
  double tmin, tmax;
  double wsum;             // sum of this lightcurve's normalised weights (1, or a band's share)
  double mm_scale;         // shared-phase: sum_k wsum_k sum_n |alpha^(k)_n|^2 (0 otherwise)
  int wmode;               // 0: sigma^-2 weights, 1: uniform (all sigma = 0)
  int status;              // FTP_LC_* bits
};

constexpr int kMaxBands = 16;         // bands of a shared-phase plan

// Statistics kernel: threads per workgroup, doubles of partials per workgroup,
// most workgroups per lightcurve.
constexpr int kStatThreads = 256;
constexpr int kStatVals = 11;
constexpr int kStatMaxBlocks = 64;

// Per-lightcurve status bits (device side).
enum : int {
  LC_BAD_INPUT = 1,        // NaN/Inf in t, y or sigma, or sigma < 0
  LC_MIXED_SIGMA = 2,      // some sigma = 0 and some > 0
  LC_ZERO_VAR = 4,         // weighted variance of y is zero
};

// Per-frequency status codes written to the caller's status array.
// option bit the per-frequency kernels read (same value as FTP_FLAG_POSITIVE_AMP)
constexpr unsigned kFlagPositiveAmp = 8u;

enum : uint8_t {
  ST_OK = 0,
  ST_DEGENERATE = 1,       // MM ~ 0 at every candidate: P = 0
  ST_CONSTANT = 2,         // p == 0: P independent of phase; theta_2 = 0 scored
  ST_NO_CONVERGE = 3,      // QR iteration limit hit (best of what was found)
  ST_BAD_LC = 4,           // the lightcurve's input was rejected
  ST_FALLBACK = 8,         // bit: the first method of the solver did not settle the pair
  ST_FALLBACK_QR = 16,     // bit: roots from the companion solve after the Aberth tier
};

template <typename R> struct PointRec;
template <> struct PointRec<float> { int cell; float frac; float2 g; };
template <> struct PointRec<double> { int cell; int pad; double frac; double2 g; };

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

// FFT work description for one pass of one grid.
struct FftGridPass {
  int64_t grid_off;        // element offset of the grid
  int64_t item_begin;      // first work item of this grid in the launch
  int64_t tile_base;       // first pass of the grid: global index of its first spreading tile
                           // (tiles that received no point were not written and read as zero);
                           // later passes: -1
  int log2n, lp, ls, lcols;  // log2 of size, pass size, stride, columns per item
};

// Solve statistics, in kCounterSlots copies: each wavefront adds to copy
// (block index mod kCounterSlots), so that the per-wave additions of a large
// grid do not all meet on one address; the host sums the copies.
constexpr int kCounterSlots = 64;
struct SolveCounters {
  unsigned long long fallback;   // frequencies the learned / uniform Newton solve did not confirm
  unsigned long long newton_iters;
  unsigned long long roots_found;
  unsigned long long qr_sweeps;
  unsigned long long aberth_iters;   // Aberth sweeps summed over solved pairs
  unsigned long long fallback_qr;    // pairs left to the companion solve after Aberth
  unsigned long long fallback_aberth;   // pairs the second Newton round left to the Aberth tier
};

}  // namespace ftp
