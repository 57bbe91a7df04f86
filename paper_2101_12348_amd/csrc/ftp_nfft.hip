// NFFT stage of the fast template periodogram on gfx950.
//
// The trig sums Z_g(m) = sum_i g_i exp(2 pi i m df (t_i - t_ref)) the method
// needs (Section 2, Eqs. CCdef-YSdef, where the paper assigns these sums to
// the NFFT; the harmonics up to 2H follow from the product-to-sum
// identities) are evaluated by Gaussian gridding
// (Dutt & Rokhlin 1993; Greengard & Lee 2004):
//   prep     : weights, weighted mean, chi^2_0 and t_ref per lightcurve; per
//              point the grid cell, fractional offset and complex strength
//              (weights modulated by exp(2 pi i m_c x) to centre the needed
//              modes), plus a tile histogram;
//   bin      : points are bucketed by spreading tile (order inside a bucket
//              is irrelevant, see below);
//   spread   : one workgroup per tile accumulates Gaussian contributions in
//              LDS as 2^60 fixed-point integers.  Integer addition is
//              associative, so the grid is bit-for-bit independent of the
//              order in which points arrive and no global atomics touch it;
//   fft      : multi-pass in-place FFT, each pass an LDS-resident radix-2
//              transform over strided columns; the output stays in mixed-radix
//              digit-reversed order, which the gather undoes by index math.
#include "ftp_internal.h"

namespace ftp {

// ------------------------------------------------------------ helpers

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = fma(a, b, -p);
}

// Reduce a double-double value to [-0.5, 0.5) and return (hi, lo).
__device__ __forceinline__ void dd_wrap_half(double& hi, double& lo) {
  double r = rint(hi);
  double h, l;
  two_sum(hi - r, lo, h, l);
  if (h >= 0.5) { h -= 1.0; }
  else if (h < -0.5) { h += 1.0; }
  hi = h; lo = l;
}

__device__ __forceinline__ int64_t find_segment(const int64_t* off, int64_t n, int64_t x) {
  // largest s in [0, n) with off[s] <= x
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ prep

// Per-lightcurve statistics: the weights (Section 1: w ~ sigma^-2 with
// sum w = 1; all sigma = 0 gives uniform weights, a mix is rejected), ybar,
// YY = chi^2_0, t_ref and the input checks. Lightcurve blockIdx.x takes
// stat_nb workgroups (blockIdx.y), a count set by its n_obs alone, so it is
// reduced in the same order alone and in a batch. Each workgroup makes two
// passes over its share of the observations: the first for the extremes, the
// counts and the sums of s and s y (s = sigma^-2; over sigma = 0 the same with
// unit weights), the second for M2_b = sum s (y - m_b)^2 around its own mean
// m_b. It writes these partials and takes a ticket. The last workgroup
// combines them in workgroup order by the pairwise update of Chan, Golub and
// LeVeque (M2 = sum_b [M2_b + W_b (m_b - m)^2]), so YY = M2 / W carries no
// one-pass cancellation. It then fills the LcInfo and resets the ticket for the
// next call.

// Block-wide sums of v[0..NS) and minima of v[NS..NS+NM) in a fixed order
// (wave shuffles, then the waves in turn); every thread receives the result.
template <int NS, int NM>
__device__ __forceinline__ void block_reduce(double* v) {
  constexpr int N = NS + NM, NW = kStatThreads / 64;
  for (int o = 32; o > 0; o >>= 1) {
    for (int q = 0; q < NS; ++q) v[q] += __shfl_xor(v[q], o);
    for (int q = NS; q < N; ++q) v[q] = fmin(v[q], __shfl_xor(v[q], o));
  }
  __shared__ double sh[NW][N];
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < N; ++q) sh[wid][q] = v[q];
  __syncthreads();
  for (int q = 0; q < N; ++q) {
    double r = sh[0][q];
    for (int k = 1; k < NW; ++k) r = q < NS ? r + sh[k][q] : fmin(r, sh[k][q]);
    v[q] = r;
  }
  __syncthreads();   // the exchange array may be reused
}

__global__ __launch_bounds__(kStatThreads) void k_prep_stats(LcInfo* lcs, const double* __restrict__ t,
                                                            const double* __restrict__ y,
                                                            const double* __restrict__ sigma, double* part,
                                                            unsigned* tickets, unsigned* zero_a, unsigned* zero_b,
                                                            int64_t n_zero) {
  // zero_a[0..n_zero) and zero_b[0..n_zero) are cleared on the way, by the
  // whole grid
  for (int64_t i = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * kStatThreads + threadIdx.x; i < n_zero;
       i += (int64_t)gridDim.x * gridDim.y * kStatThreads) {
    zero_a[i] = 0u;
    zero_b[i] = 0u;
  }
  LcInfo& L = lcs[blockIdx.x];
  const int nb = L.stat_nb;
  if ((int)blockIdx.y >= nb) return;
  unsigned* ticket = tickets + blockIdx.x;
  const int64_t b = L.obs_off, n = L.n_obs;
  const int64_t i0 = (int64_t)blockIdx.y * kStatThreads + threadIdx.x, stride = (int64_t)nb * kStatThreads;
  // W (sigma > 0), sum s y, count (sigma = 0), sum y (sigma = 0), bad; tmin, -tmax, ymin, -ymax
  double v[9] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY, INFINITY, INFINITY};
#pragma unroll 1
  for (int64_t i = i0; i < n; i += stride) {
    const double ti = t[b + i], yi = y[b + i] - L.yoff, si = sigma[b + i];
    if (!isfinite(ti) || !isfinite(yi) || !isfinite(si) || si < 0.0) v[4] = 1.0;
    if (si == 0.0) {
      v[2] += 1.0;
      v[3] += yi;
    } else {
      const double iw = 1.0 / (si * si);
      v[0] += iw;
      v[1] += iw * yi;
    }
    v[5] = fmin(v[5], ti);
    v[6] = fmin(v[6], -ti);
    v[7] = fmin(v[7], yi);
    v[8] = fmin(v[8], -yi);
  }
  block_reduce<5, 4>(v);
  const double mw = v[0] > 0.0 ? v[1] / v[0] : 0.0, mu = v[2] > 0.0 ? v[3] / v[2] : 0.0;
  double m2[2] = {0.0, 0.0};
#pragma unroll 1
  for (int64_t i = i0; i < n; i += stride) {
    const double yi = y[b + i] - L.yoff, si = sigma[b + i];
    if (si == 0.0) {
      m2[1] += (yi - mu) * (yi - mu);
    } else {
      m2[0] += (yi - mw) * (yi - mw) / (si * si);
    }
  }
  block_reduce<2, 0>(m2);
  __shared__ int last;
  if (threadIdx.x == 0) {
    double* pb = part + (L.stat_off + blockIdx.y) * kStatVals;
    for (int q = 0; q < 9; ++q) pb[q] = v[q];
    pb[9] = m2[0];
    pb[10] = m2[1];
    __threadfence();
    last = atomicAdd(ticket, 1u) == (unsigned)nb - 1u;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  // the workgroups' partials, workgroup k on thread k (nb <= kStatMaxBlocks <= kStatThreads)
  double w[9] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY, INFINITY, INFINITY};
  double bm2[2] = {0.0, 0.0};
  if ((int)threadIdx.x < nb) {
    const double* pb = part + (L.stat_off + threadIdx.x) * kStatVals;
    for (int q = 0; q < 9; ++q) w[q] = pb[q];
    bm2[0] = pb[9];
    bm2[1] = pb[10];
  }
  double mine[4] = {w[0], w[1], w[2], w[3]};
  block_reduce<5, 4>(w);
  const double tmin = w[5], tmax = -w[6], ymin = w[7], ymax = -w[8];
  const int64_t nzero = (int64_t)w[2];
  int status = 0, wmode = 0;
  double winv = 0.0, ybar = 0.0;
  if (w[4] != 0.0) status |= LC_BAD_INPUT;
  if (nzero == n) { wmode = 1; winv = 1.0 / (double)n; ybar = w[3] * winv; }
  else if (nzero > 0) status |= LC_MIXED_SIGMA;
  else { winv = 1.0 / w[0]; ybar = w[1] * winv; }
  // this workgroup's share of M2 about the whole mean
  const double wb = wmode ? mine[2] : mine[0], sb = wmode ? mine[3] : mine[1];
  const double db = wb > 0.0 ? sb / wb - ybar : 0.0;
  double m2t[1] = {status == 0 ? (wmode ? bm2[1] : bm2[0]) + wb * db * db : 0.0};
  block_reduce<1, 0>(m2t);
  if (threadIdx.x != 0) return;
  *ticket = 0u;
  const double yy = m2t[0] * winv;
  // Var(y) = 0 means every y_i is equal (rounding may leave yy slightly > 0)
  if (status == 0 && (!(yy > 0.0 && isfinite(yy)) || ymin == ymax)) status |= LC_ZERO_VAR;
  L.tref = 0.5 * (tmin + tmax);
  L.tmin = tmin;
  L.tmax = tmax;
  L.wsum = 1.0;
  L.mm_scale = 0.0;
  L.ybar = ybar;
  L.yy = yy;
  L.inv_sqrt_yy = (status == 0) ? 1.0 / sqrt(yy) : 0.0;
  L.winv = winv;
  L.wmode = wmode;
  L.status = status;
}

__device__ __forceinline__ void tile_span(int cell, int msp, int log2n, int& t0, int& t1) {
  const int n = 1 << log2n;
  const int ntile = n / kTileCells;
  int lo = cell - msp + 1;
  int hi = cell + msp;
  lo &= n - 1;   // n is a power of two
  hi &= n - 1;
  t0 = lo / kTileCells;
  t1 = hi / kTileCells;
  if (t1 == t0) t1 = -1;
  (void)ntile;
}

// Shared-phase bands (Appendix A): the per-band statistics of k_prep_stats
// combined into the object's, written back to every band so that the grids
// carry weights normalised over all bands, the common weighted mean and
// variance, and one reference time.  Band k's share of the weights is
// S_k / S with S_k = sum sigma^-2 over the band (its count with unit
// weights); ybar = sum S_k ybar_k / S; YY = sum (S_k / S)(YY_k + (ybar_k -
// ybar)^2).  A band with bad input, or bands mixing unit and sigma weights,
// reject the object; a band of constant y is fine on its own.  Band 0 also
// receives mm_scale = sum_k (S_k / S) sum_n |alpha^(k)_n|^2, the scale of the
// degeneracy test.  One thread.
__global__ void k_sp_combine(LcInfo* lcs, int n_band, const double2* alpha, int H) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int bad = 0;
  double S = 0.0, sy = 0.0, tmin = INFINITY, tmax = -INFINITY;
  for (int k = 0; k < n_band; ++k) {
    const LcInfo& L = lcs[k];
    if (L.status & (LC_BAD_INPUT | LC_MIXED_SIGMA)) bad = 1;
    if (L.wmode != lcs[0].wmode) bad = 1;
    const double Sk = 1.0 / L.winv;
    S += Sk;
    sy += Sk * L.ybar;
    tmin = fmin(tmin, L.tmin);
    tmax = fmax(tmax, L.tmax);
  }
  const double ybar = sy / S;
  double yy = 0.0, msc = 0.0;
  for (int k = 0; k < n_band; ++k) {
    const LcInfo& L = lcs[k];
    const double f = (1.0 / L.winv) / S;
    const double d = L.ybar - ybar;
    yy += f * (L.yy + d * d);
    double a2 = 0.0;
    for (int n = 0; n < H; ++n) a2 += alpha[k * H + n].x * alpha[k * H + n].x + alpha[k * H + n].y * alpha[k * H + n].y;
    msc += f * a2;
  }
  int status = bad ? LC_BAD_INPUT : 0;
  if (!bad && !(yy > 0.0 && isfinite(yy))) status = LC_ZERO_VAR;
  for (int k = 0; k < n_band; ++k) {
    LcInfo& L = lcs[k];
    const double f = (1.0 / L.winv) / S;
    L.wsum = f;
    L.winv = 1.0 / S;
    L.ybar = ybar;
    L.yy = yy;
    L.inv_sqrt_yy = status == 0 ? 1.0 / sqrt(yy) : 0.0;
    L.tref = 0.5 * (tmin + tmax);
    L.status = status;
    L.mm_scale = k == 0 ? msc : 0.0;
  }
}

// Per-workgroup aggregation of tile counts: an LDS open-addressing table keyed
// by global tile index.  A 256-point workgroup touches at most 1024 tiles (two
// grids, at most two tiles per point), so 2048 slots always leave room and a
// probe sequence ends within the table.  Counting in LDS first turns one
// global atomic per (point, tile) into one per (workgroup, tile); points in
// time order touch few tiles per workgroup.
constexpr int kTileHash = 2048;
struct TileTable {
  int key[kTileHash];
  unsigned cnt[kTileHash];
  unsigned base[kTileHash];
};

__device__ __forceinline__ void tile_table_clear(TileTable& T) {
  for (int h = threadIdx.x; h < kTileHash; h += blockDim.x) {
    T.key[h] = -1;
    T.cnt[h] = 0u;
  }
}

// Slot of `tile` (inserted if new).
__device__ __forceinline__ int tile_slot(TileTable& T, int tile) {
  unsigned h = ((unsigned)tile * 2654435761u) >> 21;   // 11-bit multiplicative hash
  for (int probe = 0; probe < kTileHash; ++probe) {
    const int old = atomicCAS(&T.key[h], -1, tile);
    if (old == -1 || old == tile) return (int)h;
    h = (h + 1u) & (kTileHash - 1);
  }
  return -1;   // not reached: the table holds at most 1024 keys
}

// Per point and grid: cell, fractional offset and modulated strength, and the
// tile histogram (counts per workgroup in LDS, then added to the global
// counts; the counts do not depend on order).
template <typename R>
__global__ __launch_bounds__(256) void k_prep_points(const LcInfo* __restrict__ lcs, int64_t n_lc,
                                                     const int64_t* __restrict__ obs_off,
                                                     int64_t n_total, const double* __restrict__ t,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ sigma,
                                                     PointRec<R>* __restrict__ pw,
                                                     PointRec<R>* __restrict__ py,
                                                     unsigned int* __restrict__ tile_count) {
  __shared__ TileTable T;
  tile_table_clear(T);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n_total) {
    const int64_t lc = find_segment(obs_off, n_lc, i);
    const LcInfo& L = lcs[lc];
    PointRec<R> recs[2];
    if (L.status != 0) {
      for (int g = 0; g < 2; ++g) { recs[g].cell = -1; recs[g].frac = 0; recs[g].g.x = 0; recs[g].g.y = 0; }
    } else {
      const double si = sigma[i];
      const double w = (L.wmode ? 1.0 : 1.0 / (si * si)) * L.winv;
      const double gval[2] = {w, w * (y[i] - L.yoff - L.ybar) * L.inv_sqrt_yy};
      // x = df (t - tref) in double-double, reduced mod 1
      double dh, dl;
      two_sum(t[i], -L.tref, dh, dl);
      double xh, xl;
      two_prod(L.df, dh, xh, xl);
      xl = fma(L.df, dl, xl);
      dd_wrap_half(xh, xl);
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int log2n = L.log2n[g];
        const double nn = (double)(1 << log2n);
        double uh = xh * nn, ul = xl * nn;   // exact scaling by a power of two
        double c = floor(uh);
        double fr = (uh - c) + ul;
        if (fr < 0.0) { fr += 1.0; c -= 1.0; }
        if (fr >= 1.0) { fr -= 1.0; c += 1.0; }
        long long ci = (long long)c;
        const long long n = 1LL << log2n;
        ci &= n - 1;   // n is a power of two
        // modulation phase frac(m_c x)
        double ph, pl;
        const double mc = (double)L.mc[g];
        two_prod(mc, xh, ph, pl);
        pl = fma(mc, xl, pl);
        dd_wrap_half(ph, pl);
        double phase = ph + pl;
        double sn, cs;
        sincospi(2.0 * phase, &sn, &cs);
        recs[g].cell = (int)ci;
        recs[g].frac = (R)fr;
        recs[g].g.x = (R)(gval[g] * cs);
        recs[g].g.y = (R)(gval[g] * sn);
        int t0, t1;
        tile_span((int)ci, L.msp, log2n, t0, t1);
        atomicAdd(&T.cnt[tile_slot(T, (int)(L.tile_base[g] + t0))], 1u);
        if (t1 >= 0) atomicAdd(&T.cnt[tile_slot(T, (int)(L.tile_base[g] + t1))], 1u);
      }
    }
    pw[i] = recs[0];
    py[i] = recs[1];
  }
  __syncthreads();
  for (int h = threadIdx.x; h < kTileHash; h += 256)
    if (T.key[h] >= 0) atomicAdd(&tile_count[T.key[h]], T.cnt[h]);
}

// Exclusive scan of 32-bit counts into 64-bit offsets, one workgroup for up
// to kScanSingleMax counts: thread k scans a contiguous run of
// ceil(n / 1024) counts; the run totals are scanned across the workgroup.
// out[n] and *total receive the sum.
__global__ __launch_bounds__(1024) void k_scan_single(const unsigned int* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ out, int64_t* __restrict__ total) {
  __shared__ int64_t sh[1024];
  const int tid = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = tid * per, e = b + per < n ? b + per : n;
  int64_t s = 0;
  for (int64_t k = b; k < e; ++k) s += in[k];
  sh[tid] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t a = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  int64_t run = sh[tid] - s;
  for (int64_t k = b; k < e; ++k) {
    out[k] = run;
    run += in[k];
  }
  if (tid == 1023) {
    out[n] = sh[1023];
    *total = sh[1023];
  }
}

// Exclusive scan of 32-bit counts into 64-bit offsets: three kernels.
__global__ __launch_bounds__(256) void k_scan_blocks(const unsigned int* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ out,
                                                     int64_t* __restrict__ block_sums) {
  __shared__ int64_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * 1024;
  int64_t v[4];
  int64_t s = 0;
  for (int k = 0; k < 4; ++k) {
    int64_t idx = base + threadIdx.x * 4 + k;
    v[k] = idx < n ? (int64_t)in[idx] : 0;
    s += v[k];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int64_t a = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += a;
    __syncthreads();
  }
  int64_t run = sh[threadIdx.x] - s;
  for (int k = 0; k < 4; ++k) {
    int64_t idx = base + threadIdx.x * 4 + k;
    if (idx < n) out[idx] = run;
    run += v[k];
  }
  if (threadIdx.x == 255) block_sums[blockIdx.x] = sh[255];
}

__global__ __launch_bounds__(256) void k_scan_sums(int64_t* __restrict__ block_sums, int64_t nb) {
  // single workgroup, sequential over chunks of 256
  __shared__ int64_t sh[256];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += 256) {
    int64_t idx = c0 + threadIdx.x;
    int64_t v = idx < nb ? block_sums[idx] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int64_t a = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += a;
      __syncthreads();
    }
    int64_t excl = sh[threadIdx.x] - v + carry;
    __syncthreads();
    if (idx < nb) block_sums[idx] = excl;
    if (threadIdx.x == 255) carry += sh[255];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t* __restrict__ out, int64_t n,
                                                  const int64_t* __restrict__ block_sums,
                                                  const unsigned int* __restrict__ in,
                                                  int64_t* __restrict__ total) {
  const int64_t base = (int64_t)blockIdx.x * 1024;
  const int64_t add = block_sums[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    int64_t idx = base + threadIdx.x * 4 + k;
    if (idx < n) {
      out[idx] += add;
      if (idx == n - 1) { out[n] = out[idx] + (int64_t)in[idx]; *total = out[n]; }
    }
  }
}

// Bucket fill: each workgroup counts its entries per tile in LDS (the entry's
// rank there comes from the LDS atomic), reserves one range per tile with a
// global atomic on the tile's cursor, and writes every entry at range start +
// rank.  The spread result does not depend on this order (exact integer
// accumulation).
template <typename R>
__global__ __launch_bounds__(256) void k_bin_fill(const LcInfo* __restrict__ lcs, int64_t n_lc,
                                                  const int64_t* __restrict__ obs_off, int64_t n_total,
                                                  const PointRec<R>* __restrict__ pw,
                                                  const PointRec<R>* __restrict__ py,
                                                  const int64_t* __restrict__ tile_off,
                                                  unsigned int* __restrict__ cursor,
                                                  int* __restrict__ bucket) {
  __shared__ TileTable T;
  tile_table_clear(T);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int slot[4], rank[4];
  int ne = 0;
  if (i < n_total) {
    const int64_t lc = find_segment(obs_off, n_lc, i);
    const LcInfo& L = lcs[lc];
    for (int g = 0; g < 2; ++g) {
      const int cell = g == 0 ? pw[i].cell : py[i].cell;
      if (cell < 0) continue;
      int t0, t1;
      tile_span(cell, L.msp, L.log2n[g], t0, t1);
      const int ts[2] = {t0, t1};
      for (int e = 0; e < 2; ++e) {
        if (ts[e] < 0) continue;
        const int h = tile_slot(T, (int)(L.tile_base[g] + ts[e]));
        slot[ne] = h;
        rank[ne] = (int)atomicAdd(&T.cnt[h], 1u) | (g << 30);
        ++ne;
      }
    }
  }
  __syncthreads();
  for (int h = threadIdx.x; h < kTileHash; h += 256)
    if (T.key[h] >= 0) T.base[h] = atomicAdd(&cursor[T.key[h]], T.cnt[h]);
  __syncthreads();
  for (int e = 0; e < ne; ++e) {
    const int h = slot[e];
    const int g = rank[e] >> 30;
    const unsigned r = (unsigned)(rank[e] & 0x3fffffff);
    bucket[tile_off[T.key[h]] + T.base[h] + r] = (int)((i << 1) | g);
  }
}

// One workgroup per tile of kTileCells cells.  Gaussian weights
// exp(-beta (cell - u)^2) for the 2 msp cells around each point; exact
// fixed-point accumulation in LDS; the tile is written once, coalesced.
template <typename R>
__global__ __launch_bounds__(256) void k_spread(const LcInfo* __restrict__ lcs, int64_t n_grids,
                                                const int64_t* __restrict__ grid_tile_base,
                                                const PointRec<R>* __restrict__ pw,
                                                const PointRec<R>* __restrict__ py,
                                                const int64_t* __restrict__ tile_off,
                                                const int* __restrict__ bucket,
                                                typename Cplx<R>::T* __restrict__ grids) {
  __shared__ unsigned long long acc[2 * kTileCells];
  const int64_t tile = blockIdx.x;
  const int64_t gi = find_segment(grid_tile_base, n_grids, tile);
  const int64_t lc = gi >> 1;
  const int g = (int)(gi & 1);
  const LcInfo& L = lcs[lc];
  const int log2n = L.log2n[g];
  const int n = 1 << log2n;
  const int cell0 = (int)(tile - L.tile_base[g]) * kTileCells;
  const int msp = L.msp;
  const R beta = (R)L.beta[g];
  const int64_t e0 = tile_off[tile], e1 = tile_off[tile + 1];
  // a tile no point reaches is not written: the first FFT pass reads it as
  // zero (with df T = 1/oversample most of each grid is such tiles)
  if (e1 == e0) return;
  for (int c = threadIdx.x; c < 2 * kTileCells; c += 256) acc[c] = 0ull;
  __syncthreads();
  const int64_t work = (e1 - e0) * (2 * msp);
  const double scale = (double)(1ull << kFixedShift);
  for (int64_t wi = threadIdx.x; wi < work; wi += 256) {
    const int64_t e = e0 + wi / (2 * msp);
    const int d = (int)(wi % (2 * msp)) - msp + 1;
    const int code = bucket[e];
    const int64_t pi = code >> 1;
    const PointRec<R> rec = (code & 1) ? py[pi] : pw[pi];
    int cell = rec.cell + d;
    cell = cell >= n ? cell - n : (cell < 0 ? cell + n : cell);
    const int local = cell - cell0;
    if (local < 0 || local >= kTileCells) continue;
    const R dist = (R)d - rec.frac;
    const R wgt = exp(-beta * dist * dist);
    const double vr = (double)(rec.g.x * wgt) * scale;
    const double vi = (double)(rec.g.y * wgt) * scale;
    atomicAdd(&acc[2 * local], (unsigned long long)llrint(vr));
    atomicAdd(&acc[2 * local + 1], (unsigned long long)llrint(vi));
  }
  __syncthreads();
  typename Cplx<R>::T* out = grids + L.grid_off[g] + cell0;
  const double inv = 1.0 / scale;
  for (int c = threadIdx.x; c < kTileCells; c += 256) {
    typename Cplx<R>::T v;
    v.x = (R)((double)(long long)acc[2 * c] * inv);
    v.y = (R)((double)(long long)acc[2 * c + 1] * inv);
    out[c] = v;
  }
}

// ------------------------------------------------------------ FFT pass

__device__ __forceinline__ void cs_pi(float x, float& s, float& c) { sincospif(x, &s, &c); }
__device__ __forceinline__ void cs_pi(double x, double& s, double& c) { sincospi(x, &s, &c); }

// One pass: for each block b and column j0 (0 <= j0 < s = 2^ls), the np-point
// transform Y[k] = sum_m x[b np s + j0 + s m] w_np^{m k} (w = e^{+2 pi i/.}),
// followed by the twiddle w_{np s}^{j0 k}; Y[k] is written back in place at
// b np s + j0 + s k.  A workgroup owns 2^lcols adjacent columns.
template <typename R>
__global__ __launch_bounds__(256) void k_fft_pass(const FftGridPass* __restrict__ passes, int64_t n_grids,
                                                  const int64_t* __restrict__ item_begin,
                                                  const typename Cplx<R>::T* __restrict__ twiddle,
                                                  typename Cplx<R>::T* __restrict__ grids,
                                                  const int64_t* __restrict__ tile_off) {
  using C = typename Cplx<R>::T;
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const int64_t item = blockIdx.x;
  const int64_t gi = find_segment(item_begin, n_grids, item);
  const FftGridPass P = passes[gi];
  const int64_t local_item = item - P.item_begin;
  const int lp = P.lp, ls = P.ls, lcols = P.lcols;
  const int np = 1 << lp, cols = 1 << lcols;
  const int64_t s = 1LL << ls;
  const int64_t groups_per_block = s >> lcols;
  const int64_t blk = local_item / groups_per_block;
  const int64_t j0b = (local_item % groups_per_block) << lcols;
  const int64_t base = blk * ((int64_t)np << ls) + j0b;   // position of element (0, 0) in the grid
  C* g = grids + P.grid_off + base;
  const int total = np << lcols;
  // load: element (m, c) -> buf[m * cols + c], eight loads in flight per
  // thread (total is a multiple of 2048 whenever it exceeds it).  The first
  // pass reads elements of spreading tiles that received no point as zero
  // (those tiles were not written); a column group (cols <= 16 adjacent
  // cells) never straddles a tile.
  const bool first = P.tile_base >= 0;
  auto in_empty_tile = [&](int64_t pos) -> bool {
    const int64_t t = P.tile_base + (pos >> kTileShift);
    return tile_off[t + 1] == tile_off[t];
  };
  const C zero = {(R)0, (R)0};
  if (total >= 8 * 256) {
    for (int e0 = threadIdx.x; e0 < total; e0 += 8 * 256) {
      C v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        const int64_t off = (int64_t)(e >> lcols) * s + (e & (cols - 1));
        v[u] = (first && in_empty_tile(base + off)) ? zero : g[off];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) buf[e0 + u * 256] = v[u];
    }
  } else {
    for (int e = threadIdx.x; e < total; e += 256) {
      const int m = e >> lcols, c = e & (cols - 1);
      const int64_t off = (int64_t)m * s + c;
      buf[e] = (first && in_empty_tile(base + off)) ? zero : g[off];
    }
  }
  __syncthreads();
  // in-place radix-2 decimation in frequency; output in bit-reversed order.
  // Pairs of stages (spans S and S/2) run as one radix-4 step per thread on
  // x[i], x[i + S/2], x[i + S], x[i + 3S/2] (i = 2S-block base + r, r < S/2):
  //   y0 = x0 + x2, y2 = (x0 - x2) w_{2S}^r, y1 = x1 + x3, y3 = (x1 - x3) w_{2S}^r i,
  //   z0 = y0 + y1, z1 = (y0 - y1) w_S^r,   z2 = y2 + y3, z3 = (y2 - y3) w_S^r,
  // exactly the two radix-2 stages (w_{2S}^{r + S/2} = w_{2S}^r i and
  // w_S^r = (w_{2S}^r)^2 taken from the table), with one LDS round trip and one
  // barrier instead of two; an odd stage count ends with one radix-2 stage.
  const int tstride = kTwiddleN >> lp;   // w_np^r = w_4096^{r * 4096/np}
  int span = np >> 1, lspan = lp - 1;
  for (; span >= 2; span >>= 2, lspan -= 2) {
    const int h = span >> 1;             // S/2
    const int ng = (np >> 2) << lcols;   // radix-4 groups per step
    for (int bi = threadIdx.x; bi < ng; bi += 256) {
      const int c = bi & (cols - 1);
      const int q = bi >> lcols;                 // 0 .. np/4 - 1
      const int r = q & (h - 1);
      const int i0 = ((q >> (lspan - 1)) << (lspan + 1)) + r;
      C x0 = buf[i0 * cols + c], x1 = buf[(i0 + h) * cols + c];
      C x2 = buf[(i0 + span) * cols + c], x3 = buf[(i0 + span + h) * cols + c];
      const C w = twiddle[(r << (lp - 1 - lspan)) * tstride];        // w_{2S}^r
      const C w2 = twiddle[(r << (lp - lspan)) * tstride];           // w_S^r
      C y0, y1, y2, y3, d;
      y0.x = x0.x + x2.x; y0.y = x0.y + x2.y;
      d.x = x0.x - x2.x; d.y = x0.y - x2.y;
      y2.x = d.x * w.x - d.y * w.y; y2.y = d.x * w.y + d.y * w.x;
      y1.x = x1.x + x3.x; y1.y = x1.y + x3.y;
      d.x = x1.x - x3.x; d.y = x1.y - x3.y;
      // (d w) i
      y3.x = -(d.x * w.y + d.y * w.x); y3.y = d.x * w.x - d.y * w.y;
      C z0, z1, z2, z3;
      z0.x = y0.x + y1.x; z0.y = y0.y + y1.y;
      d.x = y0.x - y1.x; d.y = y0.y - y1.y;
      z1.x = d.x * w2.x - d.y * w2.y; z1.y = d.x * w2.y + d.y * w2.x;
      z2.x = y2.x + y3.x; z2.y = y2.y + y3.y;
      d.x = y2.x - y3.x; d.y = y2.y - y3.y;
      z3.x = d.x * w2.x - d.y * w2.y; z3.y = d.x * w2.y + d.y * w2.x;
      buf[i0 * cols + c] = z0;
      buf[(i0 + h) * cols + c] = z1;
      buf[(i0 + span) * cols + c] = z2;
      buf[(i0 + span + h) * cols + c] = z3;
    }
    __syncthreads();
  }
  for (; span >= 1; span >>= 1, --lspan) {
    const int nb = (np >> 1) << lcols;   // butterflies per stage
    for (int bi = threadIdx.x; bi < nb; bi += 256) {
      const int c = bi & (cols - 1);
      const int q = bi >> lcols;             // 0 .. np/2-1
      const int r = q & (span - 1);
      const int i0 = ((q >> lspan) << (lspan + 1)) + r;
      const int i1 = i0 + span;
      C a = buf[i0 * cols + c], b = buf[i1 * cols + c];
      C sum, dif;
      sum.x = a.x + b.x; sum.y = a.y + b.y;
      dif.x = a.x - b.x; dif.y = a.y - b.y;
      // twiddle w_{2 span}^r = w_4096^{r * 4096/(2 span)} = w_np^{r * np/(2 span)}
      const C w = twiddle[(r << (lp - 1 - lspan)) * tstride];
      C tw;
      tw.x = dif.x * w.x - dif.y * w.y;
      tw.y = dif.x * w.y + dif.y * w.x;
      buf[i0 * cols + c] = sum;
      buf[i1 * cols + c] = tw;
    }
    __syncthreads();
  }
  // twiddle w_{np s}^{j0 k} and store Y[k] at b np s + j0 + s k
  const int log2L = lp + ls;
  for (int e = threadIdx.x; e < total; e += 256) {
    const int k = e >> lcols, c = e & (cols - 1);
    const int kr = (int)(__brev((unsigned)k) >> (32 - lp));
    C v = buf[kr * cols + c];
    if (ls > 0) {
      const int64_t j0 = j0b + c;
      const int64_t ex = (j0 * (int64_t)k) & ((1LL << log2L) - 1);
      R sn, cs;
      cs_pi((R)2.0 * (R)ex / (R)(1LL << log2L), sn, cs);
      C o;
      o.x = v.x * cs - v.y * sn;
      o.y = v.x * sn + v.y * cs;
      v = o;
    }
    g[(int64_t)k * s + c] = v;
  }
  (void)lp;
}

// Explicit instantiations.
template __global__ void k_prep_points<float>(const LcInfo*, int64_t, const int64_t*, int64_t, const double*,
                                              const double*, const double*, PointRec<float>*,
                                              PointRec<float>*, unsigned int*);
template __global__ void k_prep_points<double>(const LcInfo*, int64_t, const int64_t*, int64_t, const double*,
                                               const double*, const double*, PointRec<double>*,
                                               PointRec<double>*, unsigned int*);
template __global__ void k_bin_fill<float>(const LcInfo*, int64_t, const int64_t*, int64_t,
                                           const PointRec<float>*, const PointRec<float>*, const int64_t*,
                                           unsigned int*, int*);
template __global__ void k_bin_fill<double>(const LcInfo*, int64_t, const int64_t*, int64_t,
                                            const PointRec<double>*, const PointRec<double>*,
                                            const int64_t*, unsigned int*, int*);
template __global__ void k_spread<float>(const LcInfo*, int64_t, const int64_t*, const PointRec<float>*,
                                         const PointRec<float>*, const int64_t*, const int*, float2*);
template __global__ void k_spread<double>(const LcInfo*, int64_t, const int64_t*, const PointRec<double>*,
                                          const PointRec<double>*, const int64_t*, const int*, double2*);
template __global__ void k_fft_pass<float>(const FftGridPass*, int64_t, const int64_t*, const float2*, float2*,
                                           const int64_t*);
template __global__ void k_fft_pass<double>(const FftGridPass*, int64_t, const int64_t*, const double2*,
                                            double2*, const int64_t*);

}  // namespace ftp
