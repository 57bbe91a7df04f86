// Per-frequency companion-matrix solve (the method's root finding, Section 2:
// the zeros of Eq. finalpoly are the eigenvalues of its companion matrix,
// projected onto the unit circle and scored).
//
// One wavefront per trial frequency, persistent grid-stride loop.
//   1. gather and deconvolve the NFFT sums (or read given sums);
//   2. assemble mu (MM), eta (YM) and the trig coefficients r_d of
//      R(theta) = i psi^{-K} p(psi), K = 3H - 1;
//   3. Cayley map theta = phi0 + 2 atan(x): f(x) = (1 + x^2)^K R(theta(x)) is a
//      real polynomial of degree D = 6H - 2 whose real roots are the real
//      phases; phi0 is picked among 16 rotations to maximise |R(phi0 + pi)| (the
//      leading coefficient of f);
//   4. eigenvalues of the real companion matrix of f by Francis double-shift
//      QR (the Hessenberg matrix lives in LDS, lanes own rows or columns);
//   5. every eigenvalue is mapped back to psi, projected onto the unit circle
//      and scored (P = YM^2/(YY MM)); the best candidate is Newton-polished
//      on R(theta) and accepted only if P does not drop.
#include "ftp_solve_common.h"

namespace ftp {

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// Eigenvalues of the n x n upper Hessenberg matrix A (LDS, leading dim ld),
// EISPACK hqr structure, eigenvalues only.  Returns the number of sweeps, or
// -1 when the iteration limit is reached (remaining diagonal entries are then
// used as eigenvalue estimates).
__device__ int hqr_wave(double* A, int n, int ld, double* wr, double* wi, int lane) {
  double anorm = 0.0;
  for (int i = lane; i < n; i += 64) {
    for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) anorm += fabs(A[i * ld + j]);
  }
  anorm = wave_sum(anorm);
  if (anorm == 0.0) anorm = 1.0;
  int m = n - 1, its = 0, sweeps = 0;
  const int maxit = 30 * n;
  bool failed = false;
  while (m >= 0) {
    // largest l in [1, m] with a negligible subdiagonal, else 0
    int l = 0;
    for (int base = 0; base <= m; base += 64) {
      const int ll = base + lane;
      bool ok = false;
      if (ll >= 1 && ll <= m) {
        double s = fabs(A[(ll - 1) * ld + ll - 1]) + fabs(A[ll * ld + ll]);
        if (s == 0.0) s = anorm;
        ok = fabs(A[ll * ld + ll - 1]) <= kEps * s;
      }
      const unsigned long long mask = __ballot(ok);
      if (mask) l = base + 63 - __clzll(mask);
    }
    if (l > 0) {
      if (lane == 0) A[l * ld + l - 1] = 0.0;
    }
    __syncthreads();
    if (l == m) {
      if (lane == 0) { wr[m] = A[m * ld + m]; wi[m] = 0.0; }
      m -= 1;
      its = 0;
      __syncthreads();
      continue;
    }
    if (l == m - 1) {
      const double a = A[(m - 1) * ld + m - 1], b = A[(m - 1) * ld + m];
      const double c = A[m * ld + m - 1], d = A[m * ld + m];
      const double p = 0.5 * (a - d);
      const double q = p * p + b * c;
      if (lane == 0) {
        if (q >= 0.0) {
          double z = sqrt(q);
          z = p + copysign(z, p);
          const double e1 = d + z;
          const double e2 = z != 0.0 ? d - b * c / z : e1;
          wr[m - 1] = e1; wr[m] = e2; wi[m - 1] = 0.0; wi[m] = 0.0;
        } else {
          const double z = sqrt(-q);
          wr[m - 1] = d + p; wr[m] = d + p; wi[m - 1] = z; wi[m] = -z;
        }
      }
      m -= 2;
      its = 0;
      __syncthreads();
      continue;
    }
    if (sweeps >= maxit) { failed = true; break; }
    double S, T;
    if (its == 10 || its == 20) {
      const double s = fabs(A[m * ld + m - 1]) + fabs(A[(m - 1) * ld + m - 2]);
      const double c = A[m * ld + m] + 0.75 * s;
      S = 2.0 * c;
      T = c * c - 0.4375 * s * s;
    } else {
      S = A[(m - 1) * ld + m - 1] + A[m * ld + m];
      T = A[(m - 1) * ld + m - 1] * A[m * ld + m] - A[(m - 1) * ld + m] * A[m * ld + m - 1];
    }
    ++its;
    ++sweeps;
    double x = A[l * ld + l] * A[l * ld + l] + A[l * ld + l + 1] * A[(l + 1) * ld + l] - S * A[l * ld + l] + T;
    double y = A[(l + 1) * ld + l] * (A[l * ld + l] + A[(l + 1) * ld + l + 1] - S);
    double z = (l + 2 <= m) ? A[(l + 2) * ld + l + 1] * A[(l + 1) * ld + l] : 0.0;
    for (int k = l; k <= m - 1; ++k) {
      const bool three = k < m - 1;
      if (k > l) {
        x = A[k * ld + k - 1];
        y = A[(k + 1) * ld + k - 1];
        z = three ? A[(k + 2) * ld + k - 1] : 0.0;
      }
      const double nrm = sqrt(x * x + y * y + z * z);
      if (nrm == 0.0) continue;
      const double alpha = -copysign(nrm, x);
      const double v0 = x - alpha;
      const double v1 = y / v0, v2 = z / v0;
      const double tau = (alpha - x) / alpha;
      __syncthreads();
      if (k > l && lane == 0) {
        A[k * ld + k - 1] = alpha;
        A[(k + 1) * ld + k - 1] = 0.0;
        if (three) A[(k + 2) * ld + k - 1] = 0.0;
      }
      // rows k..k+2, columns k..m
      for (int j = k + lane; j <= m; j += 64) {
        double a0 = A[k * ld + j], a1 = A[(k + 1) * ld + j];
        double a2 = three ? A[(k + 2) * ld + j] : 0.0;
        const double w = a0 + v1 * a1 + v2 * a2;
        A[k * ld + j] = a0 - tau * w;
        A[(k + 1) * ld + j] = a1 - tau * w * v1;
        if (three) A[(k + 2) * ld + j] = a2 - tau * w * v2;
      }
      __syncthreads();
      // columns k..k+2, rows l..min(k+3, m)
      const int ihi = k + 3 < m ? k + 3 : m;
      for (int i = l + lane; i <= ihi; i += 64) {
        double a0 = A[i * ld + k], a1 = A[i * ld + k + 1];
        double a2 = three ? A[i * ld + k + 2] : 0.0;
        const double w = a0 + v1 * a1 + v2 * a2;
        A[i * ld + k] = a0 - tau * w;
        A[i * ld + k + 1] = a1 - tau * w * v1;
        if (three) A[i * ld + k + 2] = a2 - tau * w * v2;
      }
      __syncthreads();
    }
  }
  if (failed) {
    for (int i = lane; i <= m; i += 64) { wr[i] = A[i * ld + i]; wi[i] = 0.0; }
    __syncthreads();
    return -1;
  }
  return sweeps;
}

__device__ __forceinline__ size_t align2(size_t nd) { return (nd + 1) & ~(size_t)1; }

struct SolveLayout {
  double* A; double* wr; double* wi; FreqWork W; double2* hb[2]; double2* vb[2]; double* f;
};

__device__ __forceinline__ SolveLayout make_layout(double* sm, int H) {
  const int K = 3 * H - 1, D = 2 * K, n = D, ld = n + 1;
  SolveLayout s;
  double* p = sm;
  s.A = p; p += ((size_t)n * ld + 1) & ~(size_t)1;
  s.wr = p; p += ((size_t)n + 1) & ~(size_t)1;
  s.wi = p; p += ((size_t)n + 1) & ~(size_t)1;
  double2* q = reinterpret_cast<double2*>(p);
  s.W.Z = q; q += 3 * H + 1;
  s.W.mu = q; q += 2 * H + 1;
  s.W.eta = q; q += H + 1;
  s.W.r = q; q += K + 1;
  s.hb[0] = q; q += D + 1;
  s.hb[1] = q; q += D + 1;
  s.vb[0] = q; q += D + 1;
  s.vb[1] = q; q += D + 1;
  s.f = reinterpret_cast<double*>(q);
  p = s.f + (((size_t)D + 2) & ~(size_t)1);
  s.W.al = reinterpret_cast<double2*>(p);
  return s;
}

// Load the 3H sums of pair pidx (frequency index j of lightcurve L) into W.Z.
template <typename R>
__device__ __forceinline__ void load_sums(const SolveArgs& a, const LcInfo& L, int64_t pidx, int64_t j,
                                          const FreqWork& W, int lane) {
  const int H = a.H;
  if (lane == 0) W.Z[0] = make_double2(1.0, 0.0);
  if (a.sums_in) {
    for (int q = lane; q < 3 * H; q += 64) {
      const double* s = a.sums_in + (pidx * 3 * H + q) * 2;
      double2 v = make_double2(s[0], s[1]);
      if (q >= 2 * H) v = cscale(v, L.inv_sqrt_yy);
      W.Z[q + 1] = v;
    }
  } else {
    const typename Cplx<R>::T* grids = reinterpret_cast<const typename Cplx<R>::T*>(a.grids);
    for (int q = lane; q < 3 * H; q += 64) {
      const int g = q < 2 * H ? 0 : 1;
      const int k = g == 0 ? q + 1 : q - 2 * H + 1;
      W.Z[q + 1] = gather_mode<R>(L, g, (int64_t)k * j, grids);
    }
  }
  __syncthreads();
}

// Best-candidate selection across the wave: max P; near ties (1e-12 relative)
// prefer theta_1 > 0, then the smallest absolute theta_2.
struct Best { double P, th_rel, th_abs, amp_sign; int lane; };

__device__ __forceinline__ Best select_best(double P, double th_rel, double th_abs, double ym, bool valid,
                                            int lane) {
  const double pv = valid ? P : -1.0;
  const double pmax = wave_max(pv);
  const bool near = valid && pv >= pmax - 1e-12 * fmax(pmax, 1e-300);
  // key: (theta1 > 0 ? 0 : 1) * 8 + theta_abs  (theta_abs in [0, 2 pi))
  double key = near ? ((ym > 0.0 ? 0.0 : 8.0) + th_abs) : 1e30;
  double kmin = key;
  for (int o = 32; o > 0; o >>= 1) kmin = fmin(kmin, __shfl_xor(kmin, o));
  const unsigned long long mask = __ballot(near && key == kmin);
  Best b;
  b.lane = mask ? __ffsll((long long)mask) - 1 : 0;
  b.P = __shfl(pv, b.lane);
  b.th_rel = __shfl(th_rel, b.lane);
  b.th_abs = __shfl(th_abs, b.lane);
  b.amp_sign = __shfl(ym, b.lane);
  return b;
}

__device__ __forceinline__ double wrap_2pi(double x) {
  x = fmod(x, kTwoPi);
  if (x < 0.0) x += kTwoPi;
  if (x >= kTwoPi) x -= kTwoPi;
  return x;
}

// Writes the outputs for one frequency given the chosen relative phase.
__device__ __forceinline__ void write_outputs(const SolveArgs& a, const LcInfo& L, const FreqWork& W,
                                              int64_t pidx, double th_rel, double ref, uint8_t st) {
  const Cand c = eval_candidate(W, a.H, th_rel);
  const double sq = sqrt(L.yy);
  double P = c.P, amp = c.MM > 0.0 ? c.YM / c.MM * sq : 0.0;
  double off = L.ybar - c.Mbar * amp;
  double th_abs = wrap_2pi(th_rel + kTwoPi * ref);
  if (st == ST_DEGENERATE) { P = 0.0; amp = 0.0; off = L.ybar; th_abs = 0.0; }
  a.power[pidx] = P;
  a.phase[pidx] = th_abs;
  a.amp[pidx] = amp;
  a.offset[pidx] = off;
  if (a.status) a.status[pidx] = st;
}

// Degeneracy threshold: MM <= tau sum |alpha|^2 at every candidate, with tau
// set by the precision of the sums (exact sums 1e-14, FP64 NFFT 1e-9, FP32
// NFFT 1e-5: a few hundred times the sums' error relative to sum|g|).
__device__ __forceinline__ double mm_floor(const FreqWork& W, int H, double tau) {
  double s = 0.0;
  for (int n = 0; n < H; ++n) s += cabs2(W.al[n]);
  return tau * s;
}

// Scores the candidate set {theta_c} spread over lanes, polishes the best and
// writes outputs.  `valid` marks lanes holding a candidate.
__device__ __forceinline__ void finish_frequency(const SolveArgs& a, const LcInfo& L, const FreqWork& W,
                                                 int64_t pidx, double ref, double th, bool valid, uint8_t st0,
                                                 int lane) {
  const int H = a.H;
  Cand c = eval_candidate(W, H, th);
  const double floor_mm = mm_floor(W, H, a.mm_tau);
  const double mmmax = wave_max(valid ? c.MM : -1.0);
  uint8_t st = st0;
  if (mmmax <= floor_mm) st = ST_DEGENERATE;
  const bool ok = valid && c.MM > floor_mm;
  const double th_abs = wrap_2pi(th + kTwoPi * ref);
  Best b = select_best(c.P, th, th_abs, c.YM, ok || (valid && st == ST_DEGENERATE), lane);
  double best_th = b.th_rel;
  if (st != ST_DEGENERATE && st != ST_CONSTANT) {
    // Newton polish on R(theta) (all lanes redundantly); keep only if P holds
    double cur = best_th;
    double curP = eval_candidate(W, H, cur).P;
    for (int it = 0; it < 3; ++it) {
      double R, dR;
      eval_R(W, H, cur, R, dR);
      if (!(dR != 0.0) || !isfinite(R / dR)) break;
      const double nt = cur - R / dR;
      if (fabs(nt - cur) > 1e-3) break;
      const double nP = eval_candidate(W, H, nt).P;
      if (!(nP >= curP)) break;
      cur = nt;
      curP = nP;
    }
    best_th = cur;
  }
  if (lane == 0) write_outputs(a, L, W, pidx, best_th, ref, st);
}

template <typename R>
__global__ __launch_bounds__(64) void k_solve_plain(SolveArgs a) {
  extern __shared__ double sm[];
  const int lane = wave_lane();
  const int H = a.H, K = 3 * H - 1, D = 2 * K, n = D, ld = n + 1;
  SolveLayout S = make_layout(sm, H);
  const FreqWork& W = S.W;
  for (int q = lane; q < H; q += 64) S.W.al[q] = a.alpha[q];
  __syncthreads();
  int64_t total = a.total;
  if (a.list_count) total = (int64_t)*a.list_count < total ? (int64_t)*a.list_count : total;
  unsigned long long sweeps_acc = 0;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int64_t pidx = a.list ? a.list[w] : w;
    const int64_t lc = find_seg(a.freq_off, a.n_lc, pidx);
    const LcInfo& L = a.lcs[lc];
    const int64_t j = pidx - a.freq_off[lc] + 1;
    if (L.status != 0) {
      if (lane == 0) {
        a.power[pidx] = 0.0; a.phase[pidx] = 0.0; a.amp[pidx] = 0.0; a.offset[pidx] = 0.0;
        if (a.status) a.status[pidx] = ST_BAD_LC;
      }
      continue;
    }
    const double ref = ref_cycles(j, L.df, L.tref);
    load_sums<R>(a, L, pidx, j, W, lane);
    assemble_poly(W, H, lane);
    // p == 0 (R constant in theta) check
    double rmax = 0.0, mumax = 0.0, etamax = 0.0;
    for (int d = lane; d <= K; d += 64) rmax = fmax(rmax, sqrt(cabs2(W.r[d])));
    for (int e = lane; e <= 2 * H; e += 64) mumax = fmax(mumax, sqrt(cabs2(W.mu[e])));
    for (int k = lane; k <= H; k += 64) etamax = fmax(etamax, sqrt(cabs2(W.eta[k])));
    rmax = wave_max(rmax); mumax = wave_max(mumax); etamax = wave_max(etamax);
    const double rscale = mumax * etamax * (6.0 * H) * (2.0 * H + 1.0);
    if (!(rmax > 64.0 * kEps * rscale)) {
      // P does not depend on the phase: score theta_2 = 0 (absolute)
      const double th = -kTwoPi * ref;
      finish_frequency(a, L, W, pidx, ref, th, lane == 0, ST_CONSTANT, lane);
      __syncthreads();
      continue;
    }
    // rotation: maximise |R(phi0 + pi)| over 16 candidates
    double phi0 = 0.0;
    {
      double Rv = -1.0, dR;
      if (lane < 16) {
        eval_R(W, H, kTwoPi * lane / 16.0 + kPi, Rv, dR);
        Rv = fabs(Rv);
      }
      const double rm = wave_max(Rv);
      const unsigned long long mask = __ballot(lane < 16 && Rv == rm);
      const int bl = __ffsll((long long)mask) - 1;
      phi0 = kTwoPi * bl / 16.0;
    }
    // f(x) = sum_j rho_{j-K} u^j v^{2K-j}, u = 1 + i x, v = 1 - i x, rho_d = r_d e^{i d phi0};
    // homogeneous Horner h_l = u h_{l-1} + rho_{K-l} v^l.
    for (int c = lane; c <= D; c += 64) {
      double2 rk = W.r[K];
      double sn, cs;
      sincos(K * phi0, &sn, &cs);
      S.hb[0][c] = c == 0 ? cmul(rk, make_double2(cs, sn)) : make_double2(0.0, 0.0);
      S.vb[0][c] = c == 0 ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    int cur = 0;
    for (int l = 1; l <= D; ++l) {
      const int d = K - l;
      double2 rho;
      {
        const double2 rd = d >= 0 ? W.r[d] : cconj(W.r[-d]);
        double sn, cs;
        sincos(d * phi0, &sn, &cs);
        rho = cmul(rd, make_double2(cs, sn));
      }
      for (int c = lane; c <= D; c += 64) {
        const double2 vprev = c > 0 ? S.vb[cur][c - 1] : make_double2(0.0, 0.0);
        const double2 hprev = c > 0 ? S.hb[cur][c - 1] : make_double2(0.0, 0.0);
        const double2 vnew = make_double2(S.vb[cur][c].x + vprev.y, S.vb[cur][c].y - vprev.x);
        const double2 hnew = make_double2(S.hb[cur][c].x - hprev.y, S.hb[cur][c].y + hprev.x);
        S.vb[cur ^ 1][c] = vnew;
        S.hb[cur ^ 1][c] = cadd(hnew, cmul(rho, vnew));
      }
      __syncthreads();
      cur ^= 1;
    }
    for (int c = lane; c <= D; c += 64) S.f[c] = S.hb[cur][c].x;
    __syncthreads();
    // companion matrix (upper Hessenberg): row 0 = -f_{D-1-j}/f_D, subdiagonal ones
    const double lead = S.f[D];
    for (int i = lane; i < n; i += 64) {
      for (int jj = 0; jj < n; ++jj) S.A[i * ld + jj] = 0.0;
      if (i > 0) S.A[i * ld + i - 1] = 1.0;
    }
    __syncthreads();
    for (int jj = lane; jj < n; jj += 64) S.A[jj] = -S.f[D - 1 - jj] / lead;
    __syncthreads();
    const int sw = hqr_wave(S.A, n, ld, S.wr, S.wi, lane);
    uint8_t st0 = ST_OK;
    if (sw < 0) st0 = ST_NO_CONVERGE; else sweeps_acc += (unsigned long long)sw;
    // candidates: one per real eigenvalue and per complex pair (wi > 0)
    bool any = false;
    for (int base = 0; base < n; base += 64) {
      const int i = base + lane;
      double th = 0.0;
      bool valid = false;
      if (i < n) {
        const double xr = S.wr[i], xi = S.wi[i];
        if (xi >= 0.0 && isfinite(xr) && isfinite(xi)) {
          th = phi0 + atan2(xr, 1.0 - xi) + atan2(xr, 1.0 + xi);
          valid = true;
        }
      }
      (void)any;
      if (base == 0 && n <= 64) {
        finish_frequency(a, L, W, pidx, ref, th, valid, st0, lane);
      }
    }
    if (n > 64) {
      // more candidates than lanes: score in two rounds, keep the best
      double bestP = -1.0, bestTh = 0.0, bestAbs = 1e30, bestYm = 0.0;
      for (int base = 0; base < n; base += 64) {
        const int i = base + lane;
        double th = 0.0;
        bool valid = false;
        if (i < n) {
          const double xr = S.wr[i], xi = S.wi[i];
          if (xi >= 0.0 && isfinite(xr) && isfinite(xi)) {
            th = phi0 + atan2(xr, 1.0 - xi) + atan2(xr, 1.0 + xi);
            valid = true;
          }
        }
        const Cand c = eval_candidate(W, H, th);
        const double thabs = wrap_2pi(th + kTwoPi * ref);
        Best b = select_best(c.P, th, thabs, c.YM, valid && c.MM > mm_floor(W, H, a.mm_tau), lane);
        const bool better = b.P > bestP * (1.0 + 1e-12) ||
                            (b.P >= bestP * (1.0 - 1e-12) &&
                             ((b.amp_sign > 0.0 && bestYm <= 0.0) ||
                              ((b.amp_sign > 0.0) == (bestYm > 0.0) && b.th_abs < bestAbs)));
        if (better) { bestP = b.P; bestTh = b.th_rel; bestAbs = b.th_abs; bestYm = b.amp_sign; }
      }
      finish_frequency(a, L, W, pidx, ref, bestTh, lane == 0, st0, lane);
    }
    __syncthreads();
  }
  if (a.counters && lane == 0) atomicAdd(&a.counters->qr_sweeps, sweeps_acc);
}


// Writes the deconvolved sums of every pair (3H complex per pair: Z_w(k j),
// k = 1..2H, then Z_y(k j), k = 1..H with the 1/sqrt(YY) normalisation undone).
template <typename R>
__global__ __launch_bounds__(64) void k_gather_sums(SolveArgs a, double* out) {
  const int lane = wave_lane();
  const int H = a.H;
  const typename Cplx<R>::T* grids = reinterpret_cast<const typename Cplx<R>::T*>(a.grids);
  for (int64_t pidx = blockIdx.x; pidx < a.total; pidx += gridDim.x) {
    const int64_t lc = find_seg(a.freq_off, a.n_lc, pidx);
    const LcInfo& L = a.lcs[lc];
    const int64_t j = pidx - a.freq_off[lc] + 1;
    for (int q = lane; q < 3 * H; q += 64) {
      const int g = q < 2 * H ? 0 : 1;
      const int k = g == 0 ? q + 1 : q - 2 * H + 1;
      double2 v = L.status ? make_double2(0.0, 0.0) : gather_mode<R>(L, g, (int64_t)k * j, grids);
      if (g == 1) v = cscale(v, sqrt(L.yy));
      out[(pidx * 3 * H + q) * 2] = v.x;
      out[(pidx * 3 * H + q) * 2 + 1] = v.y;
    }
  }
}

// lc_stats[0..3] = t_ref, ybar, YY, status bits of the first lightcurve.
__global__ void k_export_stats(const LcInfo* lcs, double* out) {
  if (threadIdx.x == 0) {
    out[0] = lcs[0].tref;
    out[1] = lcs[0].ybar;
    out[2] = lcs[0].yy;
    out[3] = (double)lcs[0].status;
  }
}

template __global__ void k_gather_sums<float>(SolveArgs, double*);
template __global__ void k_gather_sums<double>(SolveArgs, double*);

template __global__ void k_solve_plain<float>(SolveArgs);
template __global__ void k_solve_plain<double>(SolveArgs);

}  // namespace ftp
