// Device-side pieces of the per-frequency stage shared by the companion
// solve and the learned proposal: sum gather/deconvolution, polynomial
// assembly, trig-polynomial evaluation and candidate scoring.
#pragma once

#include "ftp_internal.h"

namespace ftp {

struct SolveArgs {
  const LcInfo* lcs;
  int64_t n_lc;
  const int64_t* freq_off;       // device, n_lc + 1 (prefix of n_f)
  const int32_t* lc_block;       // optional: entry b = lightcurve of pair min(b kLcBlock, total - 1)
                                 // (b = 0..ceil(total / kLcBlock)); narrows the lightcurve search
  int64_t total;                 // number of pairs
  const void* grids;             // float2 or double2 grids
  const double* sums_in;         // optional: per pair 3H complex sums (see gather)
  const double2* alpha;          // template alpha_n, n = 1..H (shared phase: n_band x H, band-major)
  const double* ctab;            // Cayley-map table, rows j = 0..K of D + 1 doubles, D < 64 (see k_assemble)
  int n_band;                    // 0: single band; > 0: shared-phase bands (lcs[0..n_band))
  int newton_cands;              // candidates of M_FALLBACK == 0 pairs are Newton-converged roots
  int H;
  int flags;
  double mm_tau;                 // degenerate if MM <= mm_tau * sum|alpha|^2 at every candidate
  double* power;
  double* phase;
  double* amp;
  double* offset;
  uint8_t* status;
  SolveCounters* counters;   // kCounterSlots copies (counter_slot)
  unsigned* clear8;          // non-null: the assembly sets these 8 words (a chunk's queue and list counters) to 0
};

constexpr double kEps = 2.220446049250313e-16;

// Shared-memory size (bytes) of one wave's per-frequency working set.  The
// Cayley-Horner buffers (4 (D+1) complex) alias the companion matrix, which is
// only built after them.
__host__ __device__ inline size_t solve_region_a(int H) {
  const size_t D = 6 * H - 2;
  const size_t mat = D * (D + 1), hor = 8 * (D + 1);
  return ((mat > hor ? mat : hor) + 1) & ~(size_t)1;
}
__host__ __device__ inline size_t solve_lds_bytes(int H) {
  const int K = 3 * H - 1, D = 2 * K, n = D;
  size_t nd = solve_region_a(H);                    // Hessenberg matrix / Horner buffers
  nd += 2 * (((size_t)n + 1) & ~(size_t)1);         // eigenvalues (re, im)
  nd += 2 * (3 * H + 1);                            // Z
  nd += 2 * (2 * H + 1);                            // mu
  nd += 2 * (H + 1);                                // eta
  nd += 2 * (K + 1);                                // r
  nd += ((size_t)D + 2) & ~(size_t)1;               // f
  nd += 2 * H;                                      // alpha
  return nd * sizeof(double);
}
// Per-pair record in HBM passed between the assemble, root and score kernels
// (doubles): r_d (d = 0..K, complex), mu_e (e = 0..2H, complex), eta_k and
// Z_w(k) (k = 1..H, complex), meta (see the M_* slots), f_c (c = 0..D, the
// Cayley polynomial) and D root candidates theta (NaN = none).
enum : int {
  M_PHI0 = 0,      // Cayley rotation phi0
  M_REF = 1,       // frac(f_j t_ref) in cycles
  M_STATUS = 2,    // ST_* code driving the kernels
  M_LC = 3,        // lightcurve index within the chunk
  M_CANON = 4,     // canonical rotation of the network features (arg r_1)
  M_REAL_LO = 5,   // bit mask of real companion eigenvalues (low / high 32 lanes)
  M_REAL_HI = 6,
  M_FALLBACK = 7,  // 0: first method; 1: Aberth tier; 2: companion solve after Aberth
  M_WARM = 8,      // Newton roots left in the candidate slots for the next tier
  M_COUNT = 9,     // Sturm count of a frequency the first Newton round left (-1: none)
  M_REAL_X = 10,   // bit mask of real companion eigenvalues 64..95 (degree D > 64)
  M_SLOTS = 12,    // (an even count keeps f 16-byte aligned)
};
struct RecLayout {
  int K, D, r, mu, eta, zw, meta, f, cand, stride;
  __host__ __device__ explicit RecLayout(int H) {
    K = 3 * H - 1;
    D = 2 * K;
    r = 0;
    mu = r + 2 * (K + 1);
    eta = mu + 2 * (2 * H + 1);
    zw = eta + 2 * H;
    meta = zw + 2 * H;
    f = meta + M_SLOTS;
    cand = f + D + 1;
    stride = (cand + D + 3) & ~3;
  }
};

constexpr double kTwoPi = 6.283185307179586476925286766559;

// This wavefront's copy of the solve statistics.
__device__ __forceinline__ SolveCounters* counter_slot(SolveCounters* c) {
  return c + (blockIdx.x & (kCounterSlots - 1));
}
constexpr double kPi = 3.14159265358979323846264338327950288;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ int64_t find_seg_in(const int64_t* off, int64_t lo, int64_t hi, int64_t x) {
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ int64_t find_seg(const int64_t* off, int64_t n, int64_t x) {
  return find_seg_in(off, 0, n - 1, x);
}
// Lightcurve of pair x (the last one whose first pair is <= x): between the
// hint table's entries of x's block when there is one.
__device__ __forceinline__ int64_t pair_lc(const SolveArgs& a, int64_t x) {
  if (a.lc_block) {
    const int64_t b = x / kLcBlock;
    return find_seg_in(a.freq_off, a.lc_block[b], a.lc_block[b + 1], x);
  }
  return find_seg(a.freq_off, a.n_lc, x);
}

// Wavefront reductions of doubles: DPP moves inside each row of 16 lanes
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror), then
// the four row results are combined through readlane.  Every lane returns the
// same value; all 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long u = __double_as_longlong(v);
  // (every CTRL used here reads a lane of the same row: no lane is left without a source)
  const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double lane_d(double v, int src) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, src);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  return fmax(fmax(lane_d(v, 0), lane_d(v, 16)), fmax(lane_d(v, 32), lane_d(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// max |v| over the wavefront from the high words (sign cleared) of the
// doubles: the high word of |v| orders like |v|, so this is the maximum with
// its low word cleared (relative error below 2^-20, never above the maximum).
// Row stages: quad_perm [1,0,3,2], [2,3,0,1], row_half_mirror, row_mirror
// (every lane of a row ends with the row maximum); then row_bcast:15 into rows
// 1 and 3 and row_bcast:31 into rows 2 and 3 leave the maximum in lane 63.
// (DPP moves without an `old` value, so that each folds into its v_max; lanes
// of rows a row mask leaves out hold unspecified values, which do not reach
// lane 63.)
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int v) { return __builtin_amdgcn_mov_dpp(v, CTRL, ROWS, 0xf, true); }
__device__ __forceinline__ double wave_max_abs_hi(double v) {
  int h = (int)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7fffffff;
  h = max(h, dpp_i<0xB1, 0xf>(h));
  h = max(h, dpp_i<0x4E, 0xf>(h));
  h = max(h, dpp_i<0x141, 0xf>(h));
  h = max(h, dpp_i<0x140, 0xf>(h));
  h = max(h, dpp_i<0x142, 0xa>(h));
  h = max(h, dpp_i<0x143, 0xc>(h));
  h = __builtin_amdgcn_readlane(h, 63);
  return __longlong_as_double((long long)((unsigned long long)(unsigned)h << 32));
}

// Per-half maximum of |v| from the high words (as wave_max_abs_hi): the row
// stages, then row_bcast:15 into rows 1 and 3 leave the maximum of lanes
// 0..31 in lane 31 and of lanes 32..63 in lane 63.
__device__ __forceinline__ void half_max_abs_hi(double v, double& m_lo, double& m_hi) {
  int h = (int)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7fffffff;
  h = max(h, dpp_i<0xB1, 0xf>(h));
  h = max(h, dpp_i<0x4E, 0xf>(h));
  h = max(h, dpp_i<0x141, 0xf>(h));
  h = max(h, dpp_i<0x140, 0xf>(h));
  h = max(h, dpp_i<0x142, 0xa>(h));
  const int lo = __builtin_amdgcn_readlane(h, 31), hi = __builtin_amdgcn_readlane(h, 63);
  m_lo = __longlong_as_double((long long)((unsigned long long)(unsigned)lo << 32));
  m_hi = __longlong_as_double((long long)((unsigned long long)(unsigned)hi << 32));
}

// Exact per-half maximum of doubles: row stages of wave_max, then
// row_bcast:15 into rows 1 and 3; lane 31 holds the maximum of lanes 0..31,
// lane 63 that of lanes 32..63 (rows 0 and 2 end with unspecified values).
__device__ __forceinline__ void half_max_d(double v, double& m_lo, double& m_hi) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  const long long u = __double_as_longlong(v);
  const int blo = __builtin_amdgcn_mov_dpp((int)u, 0x142, 0xa, 0xf, true);
  const int bhi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0x142, 0xa, 0xf, true);
  v = fmax(v, __longlong_as_double(((long long)bhi << 32) | (long long)(unsigned)blo));
  m_lo = lane_d(v, 31);
  m_hi = lane_d(v, 63);
}

// Position of mode index q (0 <= q < n) in the digit-reversed FFT output.
__device__ __forceinline__ int64_t fft_pos(int64_t q, const LcInfo& L, int g) {
  // the pass sizes are loaded together (independent loads) before the loop
  int lps[kMaxPasses];
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) lps[p] = L.lp[g][p];
  const int npass = L.npass[g];
  int64_t pos = 0;
  int rem = L.log2n[g];
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) {
    if (p < npass) {
      const int lp = lps[p];
      rem -= lp;
      const int64_t d = q & ((1LL << lp) - 1);
      q >>= lp;
      pos += d << rem;
    }
  }
  return pos;
}

// Constant tables of the polynomial kernels below.  They are read through
// poly_table(), whose empty asm makes the pointer opaque where the function
// is used: the compiler then loads the coefficients into SGPRs at each use
// (scalar loads, kept in the scalar cache) instead of holding every
// coefficient of a loop body in a VGPR pair across the whole loop, which
// pushed the Newton kernel past its register budget.
typedef const __attribute__((address_space(4))) double* const_table;
__device__ __forceinline__ const_table poly_table(const_table t) {
  asm volatile("" : "+s"(t));
  return t;
}

// e^x for a moderate argument (|x| < 700; the deconvolution's exponents are
// below ~10): Cody-Waite reduction x = k ln 2 + r, |r| <= ln 2 / 2 (ln 2 as
// the nearest double and its remainder, each product taken in one FMA), the
// Taylor series of e^r through r^13 (truncation below 4e-18 on that
// interval), then the scaling by 2^k (the coefficients read through poly_table).
static __constant__ double kExpTab[14] = {
    1.4426950408889634074,     6.9314718055994530942e-01, 2.3190468138462996154e-17,
    1.6059043836821614599e-10, 2.0876756987868098979e-09, 2.5052108385441718775e-08,
    2.7557319223985890653e-07, 2.7557319223985890653e-06, 2.4801587301587301587e-05,
    1.9841269841269841270e-04, 1.3888888888888888889e-03, 8.3333333333333333333e-03,
    4.1666666666666666667e-02, 1.6666666666666666667e-01};
__device__ __forceinline__ double exp_small(double x) {
  const const_table T = poly_table((const_table)kExpTab);
  const double k = rint(x * T[0]);
  double r = fma(-k, T[1], x);
  r = fma(-k, T[2], r);
  double p = T[3];
#pragma unroll
  for (int i = 4; i <= 13; ++i) p = fma(p, r, T[i]);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

// Deconvolved sum Z(m) for harmonic index m on grid g (relative to t_ref;
// the y grid carries the 1/sqrt(YY) normalisation).
template <typename R>
__device__ __forceinline__ double2 gather_mode(const LcInfo& L, int g, int64_t m,
                                               const typename Cplx<R>::T* grids) {
  const int64_t n = 1LL << L.log2n[g];
  const int64_t mp = m - L.mc[g];
  const int64_t q = mp & (n - 1);   // mp mod n (n a power of two)
  const typename Cplx<R>::T v = grids[L.grid_off[g] + fft_pos(q, L, g)];
  const double fac = L.dec_a[g] * exp_small(L.dec_b[g] * (double)mp * (double)mp);
  return make_double2((double)v.x * fac, (double)v.y * fac);
}

// frac(j * df * tref) in double-double, returned in cycles [0, 1).
__device__ __forceinline__ double ref_cycles(int64_t j, double df, double tref) {
  double ah = (double)j * df;
  double al = fma((double)j, df, -ah);
  double ph = ah * tref;
  double pl = fma(ah, tref, -ph) + al * tref;
  double r = floor(ph);
  double c = (ph - r) + pl;
  c -= floor(c);
  return c;
}

// Per-frequency working set in LDS.
struct FreqWork {
  double2* Z;    // Z[0..2H] w sums (Z[0] = 1), Z[2H+1 .. 3H] y sums (k = 1..H)
  double2* mu;   // mu_e, e = 0..2H  (MM = sum_e mu_e psi^e, mu_{-e} = conj mu_e)
  double2* eta;  // eta_k, k = 0..H  (YM = sum_k eta_k psi^k, eta_0 = 0)
  double2* r;    // r_d, d = 0..K    (R(theta) = sum_d r_d psi^d, r_{-d} = conj r_d)
  double2* al;   // alpha_n at al[n-1]
};

// Assemble mu, eta, r from the sums (all lanes of one wave participate).
//   MM(psi) = sum_{n,m} a_n a_m conj(Z_{n+m} - Z_n Z_m) psi^{n+m}
//           + 2 a_n conj(a_m) conj(Z_{n-m} - Z_n conj(Z_m)) psi^{n-m} + c.c.
// (the CC~, CS~, SS~ terms of Section 2 written with Z_k = C_k + i S_k),
//   YM(psi) = sum_k a_k conj(Zy_k) psi^k + c.c.   (YC~_k = conj(Zy_k)),
//   R(theta) = 2 MM dYM/dtheta - YM dMM/dtheta = sum_d r_d psi^d,
//   r_d = i sum_k (3k - d) mu_{d-k} eta_k   (Eq. finalpoly with p = -i psi^K R).
__device__ __forceinline__ void assemble_r(const FreqWork& W, int H, int lane, double2* scr, int nl = 64);

// `scr`: LDS scratch of 8H + 2 complex values for assemble_r.  `lane` counts
// within a group of `nl` lanes working on one frequency (64: the wavefront; 32:
// a half-wave, two frequencies per wavefront); every lane of the wavefront
// calls this.
__device__ __forceinline__ void assemble_poly(const FreqWork& W, int H, int lane, double2* scr, int nl = 64) {
  for (int e = lane; e <= 2 * H; e += nl) {
    double2 acc = make_double2(0.0, 0.0);
    if (e == 0) {
      double s = 0.0;
      for (int n = 1; n <= H; ++n) s += cabs2(W.al[n - 1]) * (1.0 - cabs2(W.Z[n]));
      acc.x = 2.0 * s;
    } else {
      const int nlo = e - H > 1 ? e - H : 1;
      const int nhi = e - 1 < H ? e - 1 : H;
      for (int n = nlo; n <= nhi; ++n) {
        const int m = e - n;
        double2 t = csub(W.Z[e], cmul(W.Z[n], W.Z[m]));
        acc = cadd(acc, cmul(cmul(W.al[n - 1], W.al[m - 1]), cconj(t)));
      }
      for (int n = e + 1; n <= H; ++n) {
        const int m = n - e;
        double2 t = csub(W.Z[e], cmul(W.Z[n], cconj(W.Z[m])));
        acc = cadd(acc, cscale(cmul(cmul(W.al[n - 1], cconj(W.al[m - 1])), cconj(t)), 2.0));
      }
    }
    W.mu[e] = acc;
  }
  for (int k = lane; k <= H; k += nl) {
    W.eta[k] = k == 0 ? make_double2(0.0, 0.0) : cmul(W.al[k - 1], cconj(W.Z[2 * H + k]));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); __builtin_amdgcn_wave_barrier();
  assemble_r(W, H, lane, scr, nl);
}

// r_d, d = 0..K, of R(theta) = 2 MM dYM/dtheta - YM dMM/dtheta from the trig
// coefficients mu_e of MM and eta_k of YM (Eq. finalpoly as a trig polynomial).
// The coefficients are first laid out over their full index ranges (mu_e for
// e = -2H..4H with mu_{-e} = conj mu_e and zero beyond 2H, eta_k for k = -H..H
// with eta_0 = 0) so that the sum over k has no branches.
__device__ __forceinline__ void assemble_r(const FreqWork& W, int H, int lane, double2* scr, int nl) {
  const int K = 3 * H - 1;
  double2* mf = scr;               // mf[e + 2H], e = -2H .. 4H
  double2* ef = scr + 6 * H + 1;   // ef[k + H], k = -H .. H
  for (int i = lane; i <= 6 * H; i += nl) {
    const int e = i - 2 * H;
    mf[i] = e < 0 ? cconj(W.mu[-e]) : (e <= 2 * H ? W.mu[e] : make_double2(0.0, 0.0));
  }
  for (int i = lane; i <= 2 * H; i += nl) {
    const int k = i - H;
    ef[i] = k < 0 ? cconj(W.eta[-k]) : W.eta[k];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); __builtin_amdgcn_wave_barrier();
  for (int d = lane; d <= K; d += nl) {
    double2 acc = make_double2(0.0, 0.0);
    double s = (double)(-3 * H - d);   // 3k - d
    for (int k = -H; k <= H; ++k, s += 3.0) {
      const double2 t = cmul(mf[d - k + 2 * H], ef[k + H]);
      acc.x = fma(s, t.x, acc.x);
      acc.y = fma(s, t.y, acc.y);
    }
    W.r[d] = make_double2(-acc.y, acc.x);  // multiply by i
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); __builtin_amdgcn_wave_barrier();
}

// v from lane (lane - 1); lane 0 receives 0 (DPP wave_shr:1 with bound_ctrl:
// a lane whose source is out of range reads 0, so no zeroed `old` operand is
// needed; all lanes active)
__device__ __forceinline__ double lane_shr1(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(u & 0xffffffffull), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// v from lane (lane + 1); lane 63 receives 0 (DPP wave_shl:1)
__device__ __forceinline__ double lane_shl1(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x130, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// 1/d from the hardware estimate refined by two Newton steps (a few ulp).
__device__ __forceinline__ double fast_rcp_d(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
__host__ __device__ inline uint16_t f2bf(float x) {
  unsigned u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t b) {
  unsigned u = (unsigned)b << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}

// Network features of one pair (all 64 lanes; r: the K + 1 coefficients r_d
// of R, in LDS or global memory): the coefficients p_k,
// k = 0..D, of the phase polynomial rotated to the canonical phase (r_1 real
// and positive) and scaled to max |p_k| = 1, as (Re, Im) bf16 pairs written
// to x[2k], x[2k + 1].  p_{K+d} = -i r'_d with r'_d = r_d u^d, r'_{-d} =
// conj(r'_d) and u = e^{-i canon} = conj(r_1) / |r_1|, u^|d| by repeated
// squaring.  Returns canon = arg r_1 to single precision (0 when r_1 = 0).
__device__ __forceinline__ double pair_features(const double2* r, int K, int lane, uint16_t* x) {
  const int D = 2 * K;
  const double2 r1 = r[1];
  const double m1 = sqrt(r1.x * r1.x + r1.y * r1.y);
  // canon only maps network seeds (and training labels) between frames, where
  // Newton refines whatever it is given: single precision is enough
  const double canon = m1 > 0.0 ? (double)atan2f((float)r1.y, (float)r1.x) : 0.0;
  const double2 u = m1 > 0.0 ? make_double2(r1.x / m1, -r1.y / m1) : make_double2(1.0, 0.0);
  double2 v[2];
  double amax = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int k = lane + 64 * s;
    v[s] = make_double2(0.0, 0.0);
    if (k > D) continue;
    const int d = k - K;
    int ad = d < 0 ? -d : d;
    double2 rd = r[ad];
    double2 pw = make_double2(1.0, 0.0), b = u;
    while (ad) {
      if (ad & 1) pw = cmul(pw, b);
      b = cmul(b, b);
      ad >>= 1;
    }
    rd = cmul(rd, pw);
    if (d < 0) rd = cconj(rd);
    v[s] = make_double2(rd.y, -rd.x);   // -i (a + i b) = b - i a
    amax = fmax(amax, sqrt(v[s].x * v[s].x + v[s].y * v[s].y));
  }
  amax = wave_max(amax);
  const double sc = amax > 0.0 ? 1.0 / amax : 0.0;
  for (int s = 0; s < 2; ++s) {
    const int k = lane + 64 * s;
    if (k > D) continue;
    x[2 * k] = f2bf((float)(v[s].x * sc));
    x[2 * k + 1] = f2bf((float)(v[s].y * sc));
  }
  return canon;
}

// Work distribution of the persistent root kernels: wavefront b starts on
// item b; with a queue counter (zeroed before the launch) it then takes item
// gridDim.x + ticket when it is done, lane 0 taking the ticket with a vector
// atomic and the wave reading it from lane 0, so waves without work leave
// without touching the counter; without a counter, items are strided by the
// grid.
__device__ __forceinline__ int64_t take_ticket(unsigned* q, int lane) {
  unsigned v = 0u;
  if (lane == 0) v = atomicAdd(q, 1u);
  return (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int64_t first_item(unsigned*, int) { return (int64_t)blockIdx.x; }
__device__ __forceinline__ int64_t next_item(unsigned* q, int lane, int64_t w) {
  return q ? (int64_t)gridDim.x + take_ticket(q, lane) : w + (int64_t)gridDim.x;
}

// Candidate evaluation at relative phase theta: returns P (normalised,
// YY = 1), YM, MM and Mbar.
struct Cand { double P, YM, MM, Mbar; };

// sincos_small: 2/pi, pi/2 as a leading double and its remainder, then the
// sine series 1/17!, -1/15!, ..., -1/3! and the cosine series 1/18!, ..., -1/4!
static __constant__ double kSinCosTab[20] = {
    0.63661977236758134308,    1.5707963267948966192,     6.1232339957367660359e-17,
    2.8114572543455207632e-15, -7.6471637318198164759e-13, 1.6059043836821614599e-10,
    -2.5052108385441718775e-08, 2.7557319223985890653e-06, -1.9841269841269841270e-04,
    8.3333333333333333333e-03, -1.6666666666666666667e-01, 1.5619206968586225271e-16,
    -4.7794773323873852974e-14, 1.1470745597729724714e-11, -2.0876756987868098979e-09,
    2.7557319223985890653e-07, -2.4801587301587301587e-05, 1.3888888888888888889e-03,
    -4.1666666666666666667e-02, 0.0};

// sin and cos of a moderate angle (|x| < 2^30; every phase here is within a
// few turns of [0, 2 pi)): Cody-Waite reduction by pi/2 in two parts
// (k = rint(2x/pi), r = x - k pi/2 in [-pi/4, pi/4], the products exact in
// FMA), the Taylor series of sin and cos to r^17 and r^18 (truncation below
// 1e-19 on that interval; the coefficients are 1/n!), then the quadrant.
__device__ __forceinline__ void sincos_small(double x, double& s, double& c) {
  const const_table T = poly_table((const_table)kSinCosTab);
  const double k = rint(x * T[0]);
  double r = fma(-k, T[1], x);
  r = fma(-k, T[2], r);
  const double z = r * r;
  double ps = T[3];
#pragma unroll
  for (int i = 4; i <= 10; ++i) ps = fma(ps, z, T[i]);
  const double sr = fma(ps * z, r, r);
  double pc = T[11];
#pragma unroll
  for (int i = 12; i <= 18; ++i) pc = fma(pc, z, T[i]);
  pc = fma(pc, z, 0.5);
  const double cr = fma(-pc, z, 1.0);
  const int q = (int)k & 3;
  const double ss = (q & 1) ? cr : sr;
  const double cc = (q & 1) ? sr : cr;
  s = (q & 2) ? -ss : ss;
  c = ((q + 1) & 2) ? -cc : cc;
}

// psi b + c (complex multiply-add, four FMAs)
__device__ __forceinline__ double2 cfma(double2 b, double2 psi, double2 c) {
  return make_double2(fma(b.x, psi.x, fma(-b.y, psi.y, c.x)), fma(b.x, psi.y, fma(b.y, psi.x, c.y)));
}

// MM, YM and Mbar at theta by Horner in psi = e^{i theta}:
// MM = mu_0 + 2 Re sum_{k=1}^{2H} mu_k psi^k, YM = 2 Re sum_{k=1}^{H} eta_k psi^k,
// Mbar = 2 Re sum_{k=1}^{H} conj(W.Z[k]) psi^k, where W.Z[k] must hold the
// conjugated psi^k coefficient of Mbar, conj(alpha_k conj(Z_k)) (the scoring
// kernel converts the sums before calling).
__device__ __forceinline__ Cand eval_candidate(const FreqWork& W, int H, double theta) {
  double sn, cs;
  sincos_small(theta, sn, cs);
  const double2 psi = make_double2(cs, sn);
  double2 m = W.mu[2 * H];
  for (int k = 2 * H - 1; k >= 1; --k) m = cfma(m, psi, W.mu[k]);
  double2 y = W.eta[H], b = cconj(W.Z[H]);
  for (int k = H - 1; k >= 1; --k) {
    y = cfma(y, psi, W.eta[k]);
    b = cfma(b, psi, cconj(W.Z[k]));
  }
  // the sums above stop at psi^1: one more factor psi
  const double MM = W.mu[0].x + 2.0 * (m.x * psi.x - m.y * psi.y);
  const double YM = 2.0 * (y.x * psi.x - y.y * psi.y);
  Cand c;
  c.YM = YM;
  c.MM = MM;
  c.Mbar = 2.0 * (b.x * psi.x - b.y * psi.y);
  c.P = MM > 0.0 ? YM * YM / MM : 0.0;
  return c;
}

// R(theta) alone (Horner in psi).
__device__ __forceinline__ double eval_R_value(const FreqWork& W, int H, double theta) {
  const int K = 3 * H - 1;
  double sn, cs;
  sincos_small(theta, sn, cs);
  const double2 psi = make_double2(cs, sn);
  double2 q = W.r[K];
  for (int d = K - 1; d >= 1; --d) q = cfma(q, psi, W.r[d]);
  return W.r[0].x + 2.0 * (q.x * psi.x - q.y * psi.y);
}

// R(theta) and dR/dtheta from r_d.
__device__ __forceinline__ void eval_R(const FreqWork& W, int H, double theta, double& R, double& dR) {
  const int K = 3 * H - 1;
  double sn, cs;
  sincos_small(theta, sn, cs);
  const double2 psi = make_double2(cs, sn);
  // q(psi) = sum_{d=1}^{K} r_d psi^{d-1} and q'(psi) by Horner; with
  // p = psi q: R = r_0 + 2 Re p, dR/dtheta = -2 Im(psi p') = -2 Im(p + psi^2 q')
  double2 q = W.r[K], dq = make_double2(0.0, 0.0);
  for (int d = K - 1; d >= 1; --d) {
    dq = cfma(dq, psi, q);
    q = cfma(q, psi, W.r[d]);
  }
  const double2 p = cmul(q, psi), psi2 = cmul(psi, psi);
  R = W.r[0].x + 2.0 * p.x;
  dR = -2.0 * (p.y + (dq.x * psi2.y + dq.y * psi2.x));
}

}  // namespace ftp
