// Per-frequency stage of the fast template periodogram: the method's phase
// polynomial (Section 2, Eq. finalpoly), its roots as the eigenvalues of a
// companion matrix, and the scoring of every root (Section 2: the phase
// condition is necessary, not sufficient, so each solution is scored).
//
// Three kernels, one wavefront per trial frequency, exchanging a per-pair
// record through HBM (RecLayout):
//   k_assemble : gather and deconvolve the NFFT sums (or read given sums);
//                assemble mu (MM), eta (YM) and the trig coefficients r_d of
//                R(theta) = i psi^{-K} p(psi), K = 3H - 1; pick a rotation
//                phi0 among 16 that maximises |R(phi0 + pi)|; expand the
//                Cayley polynomial f(x) = (1 + x^2)^K R(phi0 + 2 atan x), a real
//                polynomial of degree D = 6H - 2 whose real roots are the real
//                phases (leading coefficient R(phi0 + pi));
//   k_qr<D>    : eigenvalues of the real companion matrix of f by Francis
//                double-shift QR in LDS; every eigenvalue is mapped back to
//                psi and projected onto the unit circle (a complex pair gives
//                one candidate);
//   k_score    : P = YM^2 / (YY MM) at every candidate, best by P with the
//                documented tie rule, Newton polish on R(theta) kept only if P
//                does not drop, outputs theta_2, theta_1, theta_3.
#include <hip/hip_ext.h>
#include "ftp_solve_common.h"

namespace ftp {

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// Orders this wave's LDS accesses (LDS operations of one wavefront are
// performed in program order, so a compiler fence at wavefront scope is
// enough; every workgroup here is a single wave).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Value of v in lane `src` (src must be wave-uniform).
__device__ __forceinline__ double rdlane(double v, int src) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), src);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// 1/sqrt(s) from the hardware estimate refined by two Newton steps (a few
// ulp; the Householder step is backward stable to that level).
__device__ __forceinline__ double fast_rsq(double s) {
  double y = __builtin_amdgcn_rsq(s);
  const double h = 0.5 * s;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// ------------------------------------------------------------------ QR

// f_c = sum_j rc[j] T[j][c] over the Cayley table's rows j = 0..K (column
// `col`, row stride D + 1): the table loads of eight rows are issued before
// their multiply-adds, so their latency is paid once per eight rows; the
// sums run in the order of a two-accumulator loop (even rows, odd rows).
__device__ __forceinline__ double cayley_dot(const double* rc, const double* col, int K, int D) {
  double acc0 = 0.0, acc1 = 0.0;
  int jx = 0;
  for (; jx + 7 <= K; jx += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = col[(jx + u) * (D + 1)];
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      acc0 = fma(rc[jx + u], t[u], acc0);
      acc1 = fma(rc[jx + u + 1], t[u + 1], acc1);
    }
  }
  for (; jx + 1 <= K; jx += 2) {
    acc0 = fma(rc[jx], col[jx * (D + 1)], acc0);
    acc1 = fma(rc[jx + 1], col[(jx + 1) * (D + 1)], acc1);
  }
  if (jx <= K) acc0 = fma(rc[jx], col[jx * (D + 1)], acc0);
  return acc0 + acc1;
}

// Eigenvalues of the N x N upper Hessenberg matrix A (LDS, leading dim N + 1,
// N <= 64), EISPACK hqr structure, eigenvalues only: Francis double-shift
// sweeps over the active window [l, m], deflating at negligible subdiagonals.
// Lane j owns column j in the row update of a chase step and row j in the
// column update; the next bulge column is broadcast from the updating lanes'
// registers.  Returns the number of sweeps, or -1 when the iteration limit is
// reached (the remaining diagonal entries are then used as estimates).
// Storage of the N x N upper Hessenberg matrix the QR iteration works on.
// Dense: row-major with leading dimension N + 1.  Packed: column j holds rows
// 0 .. min(j + 3, N - 1) (the Hessenberg band and the chase's bulge, which
// never leaves it) at cs(j) + i: (N - 3)(N - 4)/2 + 4 (N - 3) + 3 N doubles,
// 15 KB instead of 27 KB at N = 58, so twice as many matrices fit the LDS
// of a compute unit (the iteration is latency-bound: occupancy is its
// throughput).
template <int N>
struct DenseHess {
  double* A;
  __device__ __forceinline__ double& operator()(int i, int j) const { return A[i * (N + 1) + j]; }
};
template <int N>
struct PackedHess {
  double* P;
  __host__ __device__ static constexpr int cs(int j) {
    return ((j < N - 3 ? j : N - 3) * ((j < N - 3 ? j : N - 3) - 1)) / 2 + 4 * (j < N - 3 ? j : N - 3) +
           (j - (j < N - 3 ? j : N - 3)) * N;
  }
  __device__ __forceinline__ double& operator()(int i, int j) const { return P[cs(j) + i]; }
};

template <int N, typename Acc>
__device__ __forceinline__ int hqr_wave(const Acc& X, double* wr, double* wi, const int lane) {
  double anorm = 0.0;
  if (lane < N) {
    for (int j = (lane > 0 ? lane - 1 : 0); j < N; ++j) anorm += fabs(X(lane, j));
  }
  anorm = wave_sum(anorm);
  if (anorm == 0.0) anorm = 1.0;
  int m = N - 1, its = 0, sweeps = 0;
  constexpr int maxit = 30 * N;
  bool failed = false;
  while (m >= 0) {
    bool ok = false;
    if (lane >= 1 && lane <= m) {
      double sd = fabs(X(lane - 1, lane - 1)) + fabs(X(lane, lane));
      if (sd == 0.0) sd = anorm;
      ok = fabs(X(lane, lane - 1)) <= kEps * sd;
    }
    const unsigned long long mask = __ballot(ok);
    const int l = mask ? 63 - __clzll(mask) : 0;
    if (l == m) {
      if (lane == 0) { wr[m] = X(m, m); wi[m] = 0.0; }
      m -= 1;
      its = 0;
      continue;
    }
    if (l == m - 1) {
      const double a = X(m - 1, m - 1), b = X(m - 1, m);
      const double c = X(m, m - 1), d = X(m, m);
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
      continue;
    }
    if (sweeps >= maxit) { failed = true; break; }
    double S, T;
    const double amm = X(m, m), am1 = X(m - 1, m - 1);
    if (its == 10 || its == 20) {
      const double sx = fabs(X(m, m - 1)) + fabs(X(m - 1, m - 2));
      const double c = amm + 0.75 * sx;
      S = 2.0 * c;
      T = c * c - 0.4375 * sx * sx;
    } else {
      S = am1 + amm;
      T = am1 * amm - X(m - 1, m) * X(m, m - 1);
    }
    ++its;
    ++sweeps;
    const double all = X(l, l), al1 = X(l + 1, l);
    double x = all * all + X(l, l + 1) * al1 - S * all + T;
    double y = al1 * (all + X(l + 1, l + 1) - S);
    double z = (l + 2 <= m) ? X(l + 2, l + 1) * al1 : 0.0;
    for (int k = l; k <= m - 1; ++k) {
      const bool three = k < m - 1;
      const double s2 = x * x + y * y + z * z;
      double a0n = 0.0;
      if (s2 > 0.0) {
        const double inv = fast_rsq(s2);
        const double nrm = s2 * inv;
        const double alpha = -copysign(nrm, x);
        const double ax = fabs(x);
        const double tau = 1.0 + ax * inv;                         // (alpha - x) / alpha
        const double rv = copysign(fast_rcp_d(ax + nrm), x);        // 1 / (x - alpha)
        const double v1 = y * rv, v2 = z * rv;
        // row update: rows k..k+2, columns k..m (lane = column); the bulge
        // column k-1 becomes (alpha, 0, 0)
        if (lane >= k && lane <= m) {
          const double b0 = X(k, lane), b1 = X(k + 1, lane);
          const double b2 = three ? X(k + 2, lane) : 0.0;
          const double w = tau * (b0 + v1 * b1 + v2 * b2);
          X(k, lane) = b0 - w;
          X(k + 1, lane) = b1 - w * v1;
          if (three) X(k + 2, lane) = b2 - w * v2;
        } else if (k > l && lane == k - 1) {
          X(k, lane) = alpha;
          X(k + 1, lane) = 0.0;
          if (three) X(k + 2, lane) = 0.0;
        }
        wave_sync();
        // column update: columns k..k+2, rows l..min(k+3, m) (lane = row)
        const int ihi = k + 3 < m ? k + 3 : m;
        if (lane >= l && lane <= ihi) {
          const double c0 = X(lane, k), c1 = X(lane, k + 1);
          const double c2 = three ? X(lane, k + 2) : 0.0;
          const double w = tau * (c0 + v1 * c1 + v2 * c2);
          a0n = c0 - w;
          X(lane, k) = a0n;
          X(lane, k + 1) = c1 - w * v1;
          if (three) X(lane, k + 2) = c2 - w * v2;
        }
        wave_sync();
        if (k + 1 <= m - 1) {
          x = rdlane(a0n, k + 1);
          y = rdlane(a0n, k + 2);
          z = (k + 1 < m - 1) ? rdlane(a0n, k + 3) : 0.0;
        }
      } else if (k + 1 <= m - 1) {
        x = X(k + 1, k);
        y = X(k + 2, k);
        z = (k + 1 < m - 1) ? X(k + 3, k) : 0.0;
      }
    }
  }
  wave_sync();
  if (failed) {
    if (lane <= m) { wr[lane] = X(lane, lane); wi[lane] = 0.0; }
    wave_sync();
    return -1;
  }
  return sweeps;
}

// Balancing (Parlett & Reinsch, Numer. Math. 13 (1969); LAPACK gebal): a
// diagonal similarity by powers of 2, exact in floating point, that brings the
// off-diagonal 1-norms of each row and column within a factor of 2.  The
// companion matrix of the Cayley polynomial has entries spread over many
// orders of magnitude (binomial growth with D), and without this step the QR
// iteration loses the roots' accuracy relative to the matrix norm.
template <int N, typename Acc>
__device__ __forceinline__ void balance_wave(const Acc& X, const int lane) {
  for (int sweep = 0; sweep < 16; ++sweep) {
    bool done = true;
    for (int i = 0; i < N; ++i) {
      // off-diagonal entries of column i and row i inside the band that can
      // be nonzero (rows up to the column + 3)
      const bool off = lane < N && lane != i;
      double c = wave_sum(off && lane <= i + 3 ? fabs(X(lane, i)) : 0.0);
      const double r = wave_sum(off && i <= lane + 3 ? fabs(X(i, lane)) : 0.0);
      if (!(c > 0.0) || !(r > 0.0) || !isfinite(c) || !isfinite(r)) continue;   // (also ends the loops below)
      const double s = c + r;
      double f = 1.0, g = 0.5 * r;
      while (c < g) { f *= 2.0; c *= 4.0; }
      g = 2.0 * r;
      while (c >= g) { f *= 0.5; c *= 0.25; }
      if ((c + r) / f < 0.95 * s) {
        done = false;
        const double fi = 1.0 / f;
        if (lane < N) {
          if (i <= lane + 3) X(i, lane) *= fi;
          if (lane <= i + 3) X(lane, i) *= f;
        }
        wave_sync();
      }
    }
    if (done) break;
  }
}

// The same two steps for 64 < N <= 128 (degree D = 6H - 2 up to 88): lane j
// owns rows (columns) j and j + 64, and the bulge column is broadcast from
// whichever of the two registers holds the row.
__device__ __forceinline__ double rdlane2(double v0, double v1, int r) {
  return r < 64 ? rdlane(v0, r) : rdlane(v1, r - 64);
}

template <int N>
__device__ __forceinline__ int hqr_wave2(double* A, double* wr, double* wi, const int lane) {
  static_assert(N > 64 && N <= 128, "two rows per lane");
  constexpr int ld = N + 1;
  const int j1 = lane + 64;
  const bool has1 = j1 < N;
  double anorm = 0.0;
  for (int j = (lane > 0 ? lane - 1 : 0); j < N; ++j) anorm += fabs(A[lane * ld + j]);
  if (has1) {
    for (int j = j1 - 1; j < N; ++j) anorm += fabs(A[j1 * ld + j]);
  }
  anorm = wave_sum(anorm);
  if (anorm == 0.0) anorm = 1.0;
  int m = N - 1, its = 0, sweeps = 0;
  constexpr int maxit = 30 * N;
  bool failed = false;
  while (m >= 0) {
    bool ok0 = false, ok1 = false;
    if (lane >= 1 && lane <= m) {
      double sd = fabs(A[(lane - 1) * ld + lane - 1]) + fabs(A[lane * ld + lane]);
      if (sd == 0.0) sd = anorm;
      ok0 = fabs(A[lane * ld + lane - 1]) <= kEps * sd;
    }
    if (has1 && j1 <= m) {
      double sd = fabs(A[(j1 - 1) * ld + j1 - 1]) + fabs(A[j1 * ld + j1]);
      if (sd == 0.0) sd = anorm;
      ok1 = fabs(A[j1 * ld + j1 - 1]) <= kEps * sd;
    }
    const unsigned long long mk0 = __ballot(ok0), mk1 = __ballot(ok1);
    const int l = mk1 ? 127 - __clzll(mk1) : (mk0 ? 63 - __clzll(mk0) : 0);
    if (l == m) {
      if (lane == 0) { wr[m] = A[m * ld + m]; wi[m] = 0.0; }
      m -= 1;
      its = 0;
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
      continue;
    }
    if (sweeps >= maxit) { failed = true; break; }
    double S, T;
    const double amm = A[m * ld + m], am1 = A[(m - 1) * ld + m - 1];
    if (its == 10 || its == 20) {
      const double sx = fabs(A[m * ld + m - 1]) + fabs(A[(m - 1) * ld + m - 2]);
      const double c = amm + 0.75 * sx;
      S = 2.0 * c;
      T = c * c - 0.4375 * sx * sx;
    } else {
      S = am1 + amm;
      T = am1 * amm - A[(m - 1) * ld + m] * A[m * ld + m - 1];
    }
    ++its;
    ++sweeps;
    const double all = A[l * ld + l], al1 = A[(l + 1) * ld + l];
    double x = all * all + A[l * ld + l + 1] * al1 - S * all + T;
    double y = al1 * (all + A[(l + 1) * ld + l + 1] - S);
    double z = (l + 2 <= m) ? A[(l + 2) * ld + l + 1] * al1 : 0.0;
    for (int k = l; k <= m - 1; ++k) {
      const bool three = k < m - 1;
      const double s2 = x * x + y * y + z * z;
      double a0n[2] = {0.0, 0.0};
      if (s2 > 0.0) {
        const double inv = fast_rsq(s2);
        const double nrm = s2 * inv;
        const double alpha = -copysign(nrm, x);
        const double ax = fabs(x);
        const double tau = 1.0 + ax * inv;
        const double rv = copysign(fast_rcp_d(ax + nrm), x);
        const double v1 = y * rv, v2 = z * rv;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int j = lane + 64 * sl;
          if (j >= k && j <= m) {
            const double b0 = A[k * ld + j], b1 = A[(k + 1) * ld + j];
            const double b2 = three ? A[(k + 2) * ld + j] : 0.0;
            const double w = tau * (b0 + v1 * b1 + v2 * b2);
            A[k * ld + j] = b0 - w;
            A[(k + 1) * ld + j] = b1 - w * v1;
            if (three) A[(k + 2) * ld + j] = b2 - w * v2;
          } else if (k > l && j == k - 1) {
            A[k * ld + j] = alpha;
            A[(k + 1) * ld + j] = 0.0;
            if (three) A[(k + 2) * ld + j] = 0.0;
          }
        }
        wave_sync();
        const int ihi = k + 3 < m ? k + 3 : m;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int i = lane + 64 * sl;
          if (i >= l && i <= ihi) {
            const double c0 = A[i * ld + k], c1 = A[i * ld + k + 1];
            const double c2 = three ? A[i * ld + k + 2] : 0.0;
            const double w = tau * (c0 + v1 * c1 + v2 * c2);
            a0n[sl] = c0 - w;
            A[i * ld + k] = a0n[sl];
            A[i * ld + k + 1] = c1 - w * v1;
            if (three) A[i * ld + k + 2] = c2 - w * v2;
          }
        }
        wave_sync();
        if (k + 1 <= m - 1) {
          x = rdlane2(a0n[0], a0n[1], k + 1);
          y = rdlane2(a0n[0], a0n[1], k + 2);
          z = (k + 1 < m - 1) ? rdlane2(a0n[0], a0n[1], k + 3) : 0.0;
        }
      } else if (k + 1 <= m - 1) {
        x = A[(k + 1) * ld + k];
        y = A[(k + 2) * ld + k];
        z = (k + 1 < m - 1) ? A[(k + 3) * ld + k] : 0.0;
      }
    }
  }
  wave_sync();
  if (failed) {
    for (int i = lane; i <= m; i += 64) { wr[i] = A[i * ld + i]; wi[i] = 0.0; }
    wave_sync();
    return -1;
  }
  return sweeps;
}

template <int N>
__device__ __forceinline__ void balance_wave2(double* A, const int lane) {
  static_assert(N > 64 && N <= 128, "two rows per lane");
  constexpr int ld = N + 1;
  const int j1 = lane + 64;
  const bool has1 = j1 < N;
  for (int sweep = 0; sweep < 16; ++sweep) {
    bool done = true;
    for (int i = 0; i < N; ++i) {
      double cs = lane != i ? fabs(A[lane * ld + i]) : 0.0;
      double rs = lane != i ? fabs(A[i * ld + lane]) : 0.0;
      if (has1 && j1 != i) {
        cs += fabs(A[j1 * ld + i]);
        rs += fabs(A[i * ld + j1]);
      }
      double c = wave_sum(cs);
      const double r = wave_sum(rs);
      if (!(c > 0.0) || !(r > 0.0) || !isfinite(c) || !isfinite(r)) continue;
      const double s = c + r;
      double f = 1.0, g = 0.5 * r;
      while (c < g) { f *= 2.0; c *= 4.0; }
      g = 2.0 * r;
      while (c >= g) { f *= 0.5; c *= 0.25; }
      if ((c + r) / f < 0.95 * s) {
        done = false;
        const double fi = 1.0 / f;
        A[i * ld + lane] *= fi;
        A[lane * ld + i] *= f;
        if (has1) {
          A[i * ld + j1] *= fi;
          A[j1 * ld + i] *= f;
        }
        wave_sync();
      }
    }
    if (done) break;
  }
}

// Packed storage where the dense matrix would hold a compute unit's LDS to
// fewer than ~10 matrices (N >= 46); below, the dense layout's simpler
// addressing is faster (measured: N = 34 dense 11.5 ms, packed 12.0 ms per
// 5e4 matrices; N = 58 dense 412 ms, packed 292 ms per 3e5).
__host__ __device__ inline constexpr bool qr_packed(int N) { return N >= 46 && N <= 64; }

// doubles of the matrix storage of k_qr<N>, even so that the eigenvalue
// arrays after it stay aligned
__host__ __device__ inline size_t qr_mat_doubles(int N) {
  const int j1 = N > 3 ? N - 3 : 0;   // PackedHess<N>::cs(N)
  const size_t m = qr_packed(N) ? (size_t)((j1 * (j1 - 1)) / 2 + 4 * j1 + (N - j1) * N) : (size_t)N * (N + 1);
  return (m + 1) & ~(size_t)1;
}
__host__ __device__ inline size_t qr_lds_bytes(int D) {
  return (qr_mat_doubles(D) + 2 * (size_t)D + 2) * sizeof(double);
}

// Companion eigenvalues for the pairs of a chunk (or of a list of them).
// Candidates theta_rel (relative to t_ref) go to rec.cand; NaN marks none.
template <int N>
__global__ __launch_bounds__(64) void k_qr(double* rec, int stride, int64_t np, const int64_t* list,
                                           const unsigned int* list_count, SolveCounters* counters,
                                           unsigned* queue) {
  // the fallback tiers run beside the side stream's scoring: their waves
  // take issue priority over it on a shared SIMD (the tiers are few, latency-bound
  // waves on the step's critical path)
  __builtin_amdgcn_s_setprio(2);
  extern __shared__ double smq[];
  double* A = smq;
  double* wr = A + qr_mat_doubles(N);
  double* wi = wr + N;
  const int lane = wave_lane();
  const RecLayout RL((N + 2) / 6);
  int64_t total = np;
  if (list) total = (int64_t)*list_count;
  unsigned long long sweeps_acc = 0;
  for (int64_t w = first_item(queue, lane); w < total; w = next_item(queue, lane, w)) {
    const int64_t q = list ? list[w] : w;
    double* R = rec + q * (int64_t)stride;
    const int st = (int)R[RL.meta + M_STATUS];
    if (st == ST_BAD_LC || st == ST_CONSTANT) continue;
    const double* f = R + RL.f;
    const double lead = f[N];
    int sw;
    if constexpr (N > 64) {
      constexpr int ld = N + 1;
      for (int i = lane; i < N; i += 64) {
        for (int j = 0; j < N; ++j) A[i * ld + j] = 0.0;
        if (i > 0) A[i * ld + i - 1] = 1.0;
      }
      wave_sync();
      for (int c = lane; c < N; c += 64) A[c] = -f[N - 1 - c] / lead;
      wave_sync();
      balance_wave2<N>(A, lane);
      sw = hqr_wave2<N>(A, wr, wi, lane);
    } else {
      // the companion matrix of f: zeros, the first row, the subdiagonal of ones
      auto run = [&](const auto& X) {
        for (int q = lane; q < (int)qr_mat_doubles(N); q += 64) A[q] = 0.0;
        wave_sync();
        if (lane < N) X(0, lane) = -f[N - 1 - lane] / lead;
        if (lane >= 1 && lane < N) X(lane, lane - 1) = 1.0;
        wave_sync();
        balance_wave<N>(X, lane);
        return hqr_wave<N>(X, wr, wi, lane);
      };
      if constexpr (qr_packed(N)) sw = run(PackedHess<N>{A});
      else sw = run(DenseHess<N>{A});
    }
    if (sw < 0) {
      if (lane == 0) R[RL.meta + M_STATUS] = (double)ST_NO_CONVERGE;
    } else {
      sweeps_acc += (unsigned long long)sw;
    }
    const double phi0 = R[RL.meta + M_PHI0];
    bool real[2] = {false, false};
#pragma unroll
    for (int sl = 0; sl < (N > 64 ? 2 : 1); ++sl) {
      const int c = lane + 64 * sl;
      if (c < N) {
        const double xr = wr[c], xi = wi[c];
        double th = __longlong_as_double(0x7ff8000000000000ll);
        if (xi >= 0.0 && isfinite(xr) && isfinite(xi)) th = phi0 + atan2(xr, 1.0 - xi) + atan2(xr, 1.0 + xi);
        real[sl] = xi == 0.0 && isfinite(xr);
        R[RL.cand + c] = th;
      }
    }
    const unsigned long long rmask = __ballot(real[0]);
    const unsigned long long rmask1 = N > 64 ? __ballot(real[1]) : 0ull;
    if (lane == 0) {
      R[RL.meta + M_REAL_LO] = (double)(unsigned)(rmask & 0xffffffffull);
      R[RL.meta + M_REAL_HI] = (double)(unsigned)(rmask >> 32);
      R[RL.meta + M_REAL_X] = (double)(unsigned)(rmask1 & 0xffffffffull);
    }
    wave_sync();
  }
  if (counters && lane == 0 && sweeps_acc) atomicAdd(&counter_slot(counters)->qr_sweeps, sweeps_acc);
}

// ------------------------------------------------------------- assemble

__host__ __device__ inline size_t asm_lds_bytes(int H, int nb) {
  const int K = 3 * H - 1, D = 2 * K;
  return (size_t)(2 * ((3 * H + 1) + (2 * H + 1) + (H + 1) + (K + 1) + 4 * (D + 1) + H)) * sizeof(double) +
         (size_t)nb * (3 * H + (2 * H + 1) + H + 1) * sizeof(double2);
}

// W: per-pair work arrays; hb, vb: Horner buffers; shared phase: Zb (band
// sums, nb x 3H), T (template products, nb x (2H + 1)), alb (templates,
// nb x H), wsb (the bands' weight shares, nb).
struct AsmLayout { FreqWork W; double2* hb[2]; double2* vb[2]; double2* Zb; double2* T; double2* alb; double2* wsb; };

__device__ __forceinline__ AsmLayout asm_layout(double* sm, int H, int nb) {
  const int K = 3 * H - 1, D = 2 * K;
  AsmLayout s;
  double2* q = reinterpret_cast<double2*>(sm);
  s.W.Z = q; q += 3 * H + 1;
  s.W.mu = q; q += 2 * H + 1;
  s.W.eta = q; q += H + 1;
  s.W.r = q; q += K + 1;
  s.hb[0] = q; q += D + 1;
  s.hb[1] = q; q += D + 1;
  s.vb[0] = q; q += D + 1;
  s.vb[1] = q; q += D + 1;
  s.W.al = q; q += H;
  s.Zb = q; q += nb * 3 * H;
  s.T = q; q += nb * (2 * H + 1);
  s.alb = q; q += nb * H;
  s.wsb = q;
  return s;
}

// Compact per-frequency working set of k_assemble2 (single band, D < 64):
// Z, mu, eta, r, alpha and a scratch of max(8H + 2, K + 1) complex values
// (assemble_r's MM and YM coefficient rows; later the rotated 2 rho_j).
__host__ __device__ inline int asm2_doubles(int H) {
  const int K = 3 * H - 1;
  const int scr = 8 * H + 2 > K + 1 ? 8 * H + 2 : K + 1;
  return 2 * ((3 * H + 1) + (2 * H + 1) + (H + 1) + (K + 1) + H + scr);
}
__device__ __forceinline__ FreqWork asm2_layout(double* sm, int H, double2*& scr) {
  const int K = 3 * H - 1;
  FreqWork W;
  double2* q = reinterpret_cast<double2*>(sm);
  W.Z = q; q += 3 * H + 1;
  W.mu = q; q += 2 * H + 1;
  W.eta = q; q += H + 1;
  W.r = q; q += K + 1;
  W.al = q; q += H;
  scr = q;
  return W;
}
// Waves per workgroup of k_assemble2: they share one LDS copy of the Cayley
// table ((K + 1) (D + 1) doubles, 14 KB at H = 10), which the dot products
// read with LDS latency instead of the L2's.
constexpr int kAsmWaves = 4;
__host__ __device__ inline size_t asm2_lds_bytes(int H) {
  const int K = 3 * H - 1, D = 2 * K;
  return ((size_t)(K + 1) * (D + 1) + (size_t)kAsmWaves * 2 * asm2_doubles(H)) * sizeof(double);
}

// Shared-phase bands (Appendix A): trig coefficients of MM and YM from the
// sums of every band.  With Z^b_n (weights normalised over all bands, Z^b_0 =
// W_b the band's share) and Zy^b_n:
//   B_n = sum_b alpha^b_n conj(Z^b_n)            (psi^n coefficient of Mbar),
//   eta_n = sum_b alpha^b_n conj(Zy^b_n),
//   mu_e = sum_b conj(Z^b_e) T^b_e - C_e,
// T^b_e = sum_{n+m=e} alpha^b_n alpha^b_m + 2 sum_{n-m=e} alpha^b_n conj(alpha^b_m)
// (T^b_0 = 2 sum_n |alpha^b_n|^2) the band's sum of M^2, and C_e the same
// products of B (Mbar^2).  One band reduces to assemble_poly.  W.Z[1..H]
// receive conj(B_n), which the scoring uses with unit alpha for Mbar.
__device__ __forceinline__ void assemble_shared(const AsmLayout& S, int nb, int H, int lane) {
  const FreqWork& W = S.W;
  for (int q = lane; q < 2 * H; q += 64) {
    const int n = (q % H) + 1;
    const bool isy = q >= H;
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < nb; ++b) {
      const double2 z = S.Zb[b * 3 * H + (isy ? 2 * H + n - 1 : n - 1)];
      acc = cadd(acc, cmul(S.alb[b * H + n - 1], cconj(z)));
    }
    if (isy) W.eta[n] = acc;
    else W.Z[n] = cconj(acc);
  }
  if (lane == 0) W.eta[0] = make_double2(0.0, 0.0);
  wave_sync();
  for (int e = lane; e <= 2 * H; e += 64) {
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < nb; ++b) {
      const double2 ze = e == 0 ? S.wsb[b] : S.Zb[b * 3 * H + e - 1];
      acc = cadd(acc, cmul(cconj(ze), S.T[b * (2 * H + 1) + e]));
    }
    double2 c = make_double2(0.0, 0.0);
    if (e == 0) {
      for (int n = 1; n <= H; ++n) c.x += 2.0 * cabs2(W.Z[n]);
    } else {
      const int nlo = e - H > 1 ? e - H : 1;
      const int nhi = e - 1 < H ? e - 1 : H;
      for (int n = nlo; n <= nhi; ++n) c = cadd(c, cmul(cconj(W.Z[n]), cconj(W.Z[e - n])));
      for (int n = e + 1; n <= H; ++n) c = cadd(c, cscale(cmul(cconj(W.Z[n]), W.Z[n - e]), 2.0));
    }
    W.mu[e] = csub(acc, c);
  }
  wave_sync();
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
  wave_sync();
}

// Sums -> polynomial record for pairs [p0, p0 + np) of the chunk.
// At least four waves per SIMD (at most 128 VGPRs): the kernel is bound by
// VALU issue and latency, and the register count otherwise drifts just above 128.
template <typename R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_assemble(SolveArgs a, double* rec, int64_t p0, int64_t np) {
  extern __shared__ double sma[];
  const int lane = wave_lane();
  if (a.clear8 && blockIdx.x == 0 && lane < 8) a.clear8[lane] = 0u;
  const int H = a.H, K = 3 * H - 1, D = 2 * K;
  const RecLayout RL(H);
  const int nb = a.n_band;
  AsmLayout S = asm_layout(sma, H, nb);
  const FreqWork& W = S.W;
  if (nb == 0) {
    for (int q = lane; q < H; q += 64) S.W.al[q] = a.alpha[q];
  } else {
    for (int q = lane; q < nb * H; q += 64) S.alb[q] = a.alpha[q];
    for (int b = lane; b < nb; b += 64) S.wsb[b] = make_double2(a.lcs[b].wsum, 0.0);
    wave_sync();
    for (int q = lane; q < nb * (2 * H + 1); q += 64) {
      const int b = q / (2 * H + 1), e = q % (2 * H + 1);
      const double2* al = S.alb + b * H;
      double2 acc = make_double2(0.0, 0.0);
      if (e == 0) {
        for (int n = 0; n < H; ++n) acc.x += 2.0 * cabs2(al[n]);
      } else {
        const int nlo = e - H > 1 ? e - H : 1;
        const int nhi = e - 1 < H ? e - 1 : H;
        for (int n = nlo; n <= nhi; ++n) acc = cadd(acc, cmul(al[n - 1], al[e - n - 1]));
        for (int n = e + 1; n <= H; ++n) acc = cadd(acc, cscale(cmul(al[n - 1], cconj(al[n - e - 1])), 2.0));
      }
      S.T[q] = acc;
    }
  }
  wave_sync();
  // e^{2 pi i m / 16}, m = lane mod 16: the rotation phases d phi0 are
  // multiples of 2 pi / 16, read from here by lane index
  double tab_c, tab_s;
  sincos(kTwoPi * (lane & 15) / 16.0, &tab_s, &tab_c);
  for (int64_t w = blockIdx.x; w < np; w += gridDim.x) {
    const int64_t pidx = p0 + w;
    double* Rr = rec + w * (int64_t)RL.stride;
    const int64_t lc = pair_lc(a, pidx);
    const LcInfo& L = a.lcs[lc];
    const int64_t j = pidx - a.freq_off[lc] + 1;
    if (L.status != 0) {
      if (lane == 0) {
        Rr[RL.meta + M_STATUS] = (double)ST_BAD_LC;
        Rr[RL.meta + M_LC] = (double)lc;
        Rr[RL.meta + M_FALLBACK] = 0.0;
        Rr[RL.meta + M_WARM] = 0.0;
      }
      continue;
    }
    const double ref = ref_cycles(j, L.df, L.tref);
    if (nb == 0) {
      load_sums<R>(a, L, pidx, j, W, lane);
      assemble_poly(W, H, lane, S.hb[0]);
    } else {
      // every band's sums of this frequency (grids of lightcurves 0..nb-1)
      const typename Cplx<R>::T* grids = reinterpret_cast<const typename Cplx<R>::T*>(a.grids);
      for (int q = lane; q < nb * 3 * H; q += 64) {
        const int b = q / (3 * H), qq = q % (3 * H);
        const int g = qq < 2 * H ? 0 : 1;
        const int k = g == 0 ? qq + 1 : qq - 2 * H + 1;
        S.Zb[q] = gather_mode<R>(a.lcs[b], g, (int64_t)k * j, grids);
      }
      wave_sync();
      assemble_shared(S, nb, H, lane);
      assemble_r(W, H, lane, S.hb[0]);
    }
    double rmax = 0.0, mumax = 0.0, etamax = 0.0;
    // (largest squared magnitudes, one square root each: sqrt is monotone and
    // correctly rounded, so this is the largest magnitude)
    for (int d = lane; d <= K; d += 64) rmax = fmax(rmax, cabs2(W.r[d]));
    for (int e = lane; e <= 2 * H; e += 64) mumax = fmax(mumax, cabs2(W.mu[e]));
    for (int k = lane; k <= H; k += 64) etamax = fmax(etamax, cabs2(W.eta[k]));
    rmax = sqrt(rmax);
    mumax = sqrt(mumax);
    etamax = sqrt(etamax);
    // maxima from the doubles' high words (within 2^-20): the threshold
    // below only separates R = 0 from rounding noise
    rmax = wave_max_abs_hi(rmax);
    mumax = wave_max_abs_hi(mumax);
    etamax = wave_max_abs_hi(etamax);
    const double rscale = mumax * etamax * (6.0 * H) * (2.0 * H + 1.0);
    const bool constant = !(rmax > 64.0 * kEps * rscale);
    double phi0 = 0.0;
    if (!constant) {
      double Rv = -1.0;
      if (lane < 16) Rv = fabs(eval_R_value(W, H, kTwoPi * lane / 16.0 + kPi));
      const double rm = wave_max(Rv);
      const unsigned long long mask = __ballot(lane < 16 && Rv == rm);
      const int k0 = __ffsll((long long)mask) - 1;
      phi0 = kTwoPi * k0 / 16.0;
      // f(x) = sum_j rho_{j-K} u^j v^{2K-j}, u = 1 + i x, v = 1 - i x,
      // rho_d = r_d e^{i d phi0}; homogeneous Horner h_l = u h_{l-1} + rho_{K-l} v^l
      const double cK = rdlane(tab_c, (K * k0) & 15), sK = rdlane(tab_s, (K * k0) & 15);
      if (D < 64) {
        // f_c = sum_j (rho_{j-K}.x or .y) T[j][c] with the Cayley-map table
        // (coefficient c of u^j v^(D-j), u = 1 + i x, v = 1 - i x, divided by
        // i^c), whose terms j and D - j are equal (the table keeps rows j <=
        // K): f_c = sum_{j<K} 2 rho'_j T[j][c] + rho'_K T[K][c].  Lane j forms
        // 2 rho_{j-K} (rho_0 once), lane c the dot product of column c.
        double* rx = reinterpret_cast<double*>(S.hb[0]);
        double* ry = rx + (K + 1);
        {
          const int d = lane - K;
          const double ec = __shfl(tab_c, (d * k0) & 15), es = __shfl(tab_s, (d * k0) & 15);
          if (lane <= K) {
            const double2 rho = cmul(cconj(W.r[-d]), make_double2(ec, es));
            const double wgt = lane < K ? 2.0 : 1.0;
            rx[lane] = wgt * rho.x;
            ry[lane] = wgt * rho.y;
          }
        }
        wave_sync();
        if (lane <= D) {
          const double* rc = (lane & 1) ? ry : rx;
          Rr[RL.f + lane] = cayley_dot(rc, a.ctab + lane, K, D);
        }
      } else {
        for (int c = lane; c <= D; c += 64) {
          S.hb[0][c] = c == 0 ? cmul(W.r[K], make_double2(cK, sK)) : make_double2(0.0, 0.0);
          S.vb[0][c] = c == 0 ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
        }
        wave_sync();
        for (int l = 1; l <= D; ++l) {
          const int d = K - l;
          const double2 rd = d >= 0 ? W.r[d] : cconj(W.r[-d]);
          const int m = (d * k0) & 15;
          const double2 rho = cmul(rd, make_double2(rdlane(tab_c, m), rdlane(tab_s, m)));
          const double2* hsrc = (l & 1) ? S.hb[0] : S.hb[1];
          const double2* vsrc = (l & 1) ? S.vb[0] : S.vb[1];
          double2* hdst = (l & 1) ? S.hb[1] : S.hb[0];
          double2* vdst = (l & 1) ? S.vb[1] : S.vb[0];
          for (int c = lane; c <= D; c += 64) {
            const double2 vprev = c > 0 ? vsrc[c - 1] : make_double2(0.0, 0.0);
            const double2 hprev = c > 0 ? hsrc[c - 1] : make_double2(0.0, 0.0);
            const double2 vnew = make_double2(vsrc[c].x + vprev.y, vsrc[c].y - vprev.x);
            const double2 hnew = make_double2(hsrc[c].x - hprev.y, hsrc[c].y + hprev.x);
            vdst[c] = vnew;
            hdst[c] = cadd(hnew, cmul(rho, vnew));
          }
          wave_sync();
        }
        const double2* hfin = (D & 1) ? S.hb[1] : S.hb[0];
        for (int c = lane; c <= D; c += 64) Rr[RL.f + c] = hfin[c].x;
      }
    }
    for (int d = lane; d <= K; d += 64) { Rr[RL.r + 2 * d] = W.r[d].x; Rr[RL.r + 2 * d + 1] = W.r[d].y; }
    for (int e = lane; e <= 2 * H; e += 64) { Rr[RL.mu + 2 * e] = W.mu[e].x; Rr[RL.mu + 2 * e + 1] = W.mu[e].y; }
    for (int k = lane; k < H; k += 64) {
      Rr[RL.eta + 2 * k] = W.eta[k + 1].x;
      Rr[RL.eta + 2 * k + 1] = W.eta[k + 1].y;
      Rr[RL.zw + 2 * k] = W.Z[k + 1].x;
      Rr[RL.zw + 2 * k + 1] = W.Z[k + 1].y;
    }
    if (lane == 0) {
      Rr[RL.meta + M_PHI0] = phi0;
      Rr[RL.meta + M_REF] = ref;
      Rr[RL.meta + M_STATUS] = constant ? (double)ST_CONSTANT : (double)ST_OK;
      Rr[RL.meta + M_LC] = (double)lc;
      Rr[RL.meta + M_FALLBACK] = 0.0;
      Rr[RL.meta + M_WARM] = 0.0;
    }
    wave_sync();
  }
}

// Two frequencies per wavefront (single band, sums from the grids, D < 64):
// frequencies 2b and 2b + 1 of the chunk on lanes 0..31 and 32..63, each half
// with its own LDS working set.  The assembly's per-frequency loops have 3H,
// 2H + 1, K + 1 or 16 lanes of work, which a half-wave holds, so one
// instruction stream serves two frequencies; the Cayley dot products (D + 1
// columns) take two rounds of 32.  Maxima and the rotation argmax are reduced
// per half (row broadcast into lanes 31 and 63).  A pair with status
// "constant" or from a rejected lightcurve still runs the (cheap) rotation and
// dot products of its half, whose results are not written.
template <typename R>
__global__ __launch_bounds__(64 * kAsmWaves) __attribute__((amdgpu_waves_per_eu(4))) void k_assemble2(SolveArgs a, double* rec,
                                                                                          int64_t p0, int64_t np) {
  extern __shared__ double sma[];
  const int lane = wave_lane(), half = lane >> 5, hl = lane & 31, wv = threadIdx.x >> 6;
  if (a.clear8 && blockIdx.x == 0 && threadIdx.x < 8) a.clear8[threadIdx.x] = 0u;
  const int H = a.H, K = 3 * H - 1, D = 2 * K;
  const RecLayout RL(H);
  // the Cayley table, shared by the workgroup's waves
  double* ctab = sma;
  const int ntab = (K + 1) * (D + 1);
  for (int i = threadIdx.x; i < ntab; i += 64 * kAsmWaves) ctab[i] = a.ctab[i];
  double2* scr;
  const FreqWork W = asm2_layout(sma + ntab + (2 * wv + half) * asm2_doubles(H), H, scr);
  for (int q = hl; q < H; q += 32) W.al[q] = a.alpha[q];
  __syncthreads();
  double tab_c, tab_s;
  sincos(kTwoPi * (lane & 15) / 16.0, &tab_s, &tab_c);
  const typename Cplx<R>::T* grids = reinterpret_cast<const typename Cplx<R>::T*>(a.grids);
  const int64_t gw = (int64_t)blockIdx.x * kAsmWaves + wv, nw = (int64_t)gridDim.x * kAsmWaves;
  for (int64_t w0 = 2 * gw; w0 < np; w0 += 2 * nw) {
    const bool has = w0 + half < np;                    // an empty second half repeats the first
    const int64_t w = has ? w0 + half : w0;
    const int64_t pidx = p0 + w;
    double* Rr = rec + w * (int64_t)RL.stride;
    const int64_t lc = pair_lc(a, pidx);
    const LcInfo& L = a.lcs[lc];
    const int64_t j = pidx - a.freq_off[lc] + 1;
    const bool bad = L.status != 0;
    if (hl == 0) W.Z[0] = make_double2(1.0, 0.0);
    for (int q = hl; q < 3 * H; q += 32) {
      const int g = q < 2 * H ? 0 : 1;
      const int k = g == 0 ? q + 1 : q - 2 * H + 1;
      W.Z[q + 1] = bad ? make_double2(0.0, 0.0) : gather_mode<R>(L, g, (int64_t)k * j, grids);
    }
    wave_sync();
    assemble_poly(W, H, hl, scr, 32);
    const double ref = ref_cycles(j, L.df, L.tref);
    double rmax = 0.0, mumax = 0.0, etamax = 0.0;
    for (int d = hl; d <= K; d += 32) rmax = fmax(rmax, cabs2(W.r[d]));
    for (int e = hl; e <= 2 * H; e += 32) mumax = fmax(mumax, cabs2(W.mu[e]));
    for (int k = hl; k <= H; k += 32) etamax = fmax(etamax, cabs2(W.eta[k]));
    rmax = sqrt(rmax);
    mumax = sqrt(mumax);
    etamax = sqrt(etamax);
    {
      double lo, hi;
      half_max_abs_hi(rmax, lo, hi);
      rmax = half ? hi : lo;
      half_max_abs_hi(mumax, lo, hi);
      mumax = half ? hi : lo;
      half_max_abs_hi(etamax, lo, hi);
      etamax = half ? hi : lo;
    }
    const double rscale = mumax * etamax * (6.0 * H) * (2.0 * H + 1.0);
    const bool constant = !(rmax > 64.0 * kEps * rscale);
    // rotation phi0: the 16 candidates of each half on its lanes 0..15
    double Rv = -1.0;
    if (hl < 16) Rv = fabs(eval_R_value(W, H, kTwoPi * hl / 16.0 + kPi));
    double rm;
    {
      double lo, hi;
      half_max_d(Rv, lo, hi);
      rm = half ? hi : lo;
    }
    const unsigned long long mask = __ballot(hl < 16 && Rv == rm);
    const unsigned hm = half ? (unsigned)(mask >> 32) : (unsigned)mask;
    const int k0 = hm ? __ffs(hm) - 1 : 0;
    const double phi0 = constant ? 0.0 : kTwoPi * k0 / 16.0;
    // 2 rho_j = 2 r_{j-K} e^{i (j-K) phi0}, j = 0..K - 1, and rho_K (K + 1 <=
    // 30 lanes: every lane takes part in the table reads), then the dot
    // products over the table's rows j <= K (the terms j and D - j are equal)
    double* rx = reinterpret_cast<double*>(scr);
    double* ry = rx + (K + 1);
    {
      const int jx = hl, d = jx - K;
      const int m = (d * k0) & 15;
      const double ec = __shfl(tab_c, m), es = __shfl(tab_s, m);
      if (jx <= K) {
        const double2 rho = cmul(cconj(W.r[-d]), make_double2(ec, es));
        const double wgt = jx < K ? 2.0 : 1.0;
        rx[jx] = wgt * rho.x;
        ry[jx] = wgt * rho.y;
      }
    }
    wave_sync();
    const bool write = has && !bad;
    for (int c = hl; c <= D; c += 32) {
      const double* rc = (c & 1) ? ry : rx;
      const double fc = cayley_dot(rc, ctab + c, K, D);
      if (write && !constant) Rr[RL.f + c] = fc;
    }
    if (write) {
      for (int d = hl; d <= K; d += 32) { Rr[RL.r + 2 * d] = W.r[d].x; Rr[RL.r + 2 * d + 1] = W.r[d].y; }
      for (int e = hl; e <= 2 * H; e += 32) { Rr[RL.mu + 2 * e] = W.mu[e].x; Rr[RL.mu + 2 * e + 1] = W.mu[e].y; }
      for (int k = hl; k < H; k += 32) {
        Rr[RL.eta + 2 * k] = W.eta[k + 1].x;
        Rr[RL.eta + 2 * k + 1] = W.eta[k + 1].y;
        Rr[RL.zw + 2 * k] = W.Z[k + 1].x;
        Rr[RL.zw + 2 * k + 1] = W.Z[k + 1].y;
      }
      if (hl == 0) {
        Rr[RL.meta + M_PHI0] = phi0;
        Rr[RL.meta + M_REF] = ref;
        Rr[RL.meta + M_STATUS] = constant ? (double)ST_CONSTANT : (double)ST_OK;
        Rr[RL.meta + M_LC] = (double)lc;
        Rr[RL.meta + M_FALLBACK] = 0.0;
        Rr[RL.meta + M_WARM] = 0.0;
      }
    } else if (has && hl == 0) {
      Rr[RL.meta + M_STATUS] = (double)ST_BAD_LC;
      Rr[RL.meta + M_LC] = (double)lc;
      Rr[RL.meta + M_FALLBACK] = 0.0;
      Rr[RL.meta + M_WARM] = 0.0;
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------- score

// Best-candidate selection across the wave: max P; near ties (1e-12 relative)
// prefer theta_1 > 0, then the smallest absolute theta_2.
struct Best { double P, th_rel, th_abs, amp_sign; int lane; };

__device__ __forceinline__ Best select_best(double P, double th_rel, double th_abs, double ym, bool valid,
                                            int lane) {
  const double pv = valid ? P : -1.0;
  const double pmax = wave_max(pv);
  const bool near = valid && pv >= pmax - 1e-12 * fmax(pmax, 1e-300);
  double key = near ? ((ym > 0.0 ? 0.0 : 8.0) + th_abs) : 1e30;
  const double kmin = -wave_max(-key);
  const unsigned long long mask = __ballot(near && key == kmin);
  Best b;
  b.lane = mask ? __ffsll((long long)mask) - 1 : 0;
  b.P = __shfl(pv, b.lane);
  b.th_rel = __shfl(th_rel, b.lane);
  b.th_abs = __shfl(th_abs, b.lane);
  b.amp_sign = __shfl(ym, b.lane);
  return b;
}

// select_best over two candidates per lane (candidate c = lane + 64 slot,
// degree D > 64); `slot` receives the winner's slot, Best.lane its lane.
__device__ __forceinline__ Best select_best2(const double (&P)[2], const double (&th_rel)[2],
                                             const double (&th_abs)[2], const double (&ym)[2],
                                             const bool (&valid)[2], int& slot) {
  const double p0 = valid[0] ? P[0] : -1.0, p1 = valid[1] ? P[1] : -1.0;
  const double pmax = wave_max(fmax(p0, p1));
  const double lo = pmax - 1e-12 * fmax(pmax, 1e-300);
  const bool n0 = valid[0] && p0 >= lo, n1 = valid[1] && p1 >= lo;
  const double k0 = n0 ? ((ym[0] > 0.0 ? 0.0 : 8.0) + th_abs[0]) : 1e30;
  const double k1 = n1 ? ((ym[1] > 0.0 ? 0.0 : 8.0) + th_abs[1]) : 1e30;
  const double kmin = -wave_max(-fmin(k0, k1));
  const unsigned long long m0 = __ballot(n0 && k0 == kmin), m1 = __ballot(n1 && k1 == kmin);
  slot = m0 ? 0 : (m1 ? 1 : 0);
  const unsigned long long mask = m0 ? m0 : m1;
  Best b;
  b.lane = mask ? __ffsll((long long)mask) - 1 : 0;
  b.P = slot ? __shfl(p1, b.lane) : __shfl(p0, b.lane);
  b.th_rel = slot ? __shfl(th_rel[1], b.lane) : __shfl(th_rel[0], b.lane);
  b.th_abs = slot ? __shfl(th_abs[1], b.lane) : __shfl(th_abs[0], b.lane);
  b.amp_sign = slot ? __shfl(ym[1], b.lane) : __shfl(ym[0], b.lane);
  return b;
}

__device__ __forceinline__ double wrap_2pi(double x) {
  x = fmod(x, kTwoPi);
  if (x < 0.0) x += kTwoPi;
  if (x >= kTwoPi) x -= kTwoPi;
  return x;
}

// Degeneracy threshold: MM <= tau sum |alpha|^2 at every candidate, with tau
// set by the precision of the sums (exact sums 1e-14, FP64 NFFT 1e-9, FP32
// NFFT 1e-5: a few hundred times the sums' error relative to sum|g|).
__device__ __forceinline__ double mm_floor(const FreqWork& W, int H, double tau) {
  double s = 0.0;
  for (int n = 0; n < H; ++n) s += cabs2(W.al[n]);
  return tau * s;
}

__host__ __device__ inline size_t score_lds_bytes(int H) {
  const int K = 3 * H - 1;
  return (size_t)(2 * ((3 * H + 1) + (2 * H + 1) + (H + 1) + (K + 1) + H)) * sizeof(double);
}

// Scores all candidates of pairs [p0, p0 + np) and writes the outputs.  At
// least four waves per SIMD (at most 128 VGPRs, no spills; measured faster
// than five waves with spills, or than the uncapped allocation).
// `list` (device, *list_n entries): score only those pairs of the chunk.
// NSL: candidates per lane (2 for degree D > 64).
template <int NSL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_score(SolveArgs a, const double* rec, int64_t p0, int64_t np,
                                                                                      const int64_t* list,
                                                                                      const unsigned* list_n) {
  // the fallback tiers run beside the side stream's scoring: their waves
  // take issue priority over it on a shared SIMD (the tiers are few, latency-bound
  // waves on the step's critical path)
  __builtin_amdgcn_s_setprio(2);
  extern __shared__ double sms[];
  const int lane = wave_lane();
  const int H = a.H, K = 3 * H - 1, D = 2 * K;
  const RecLayout RL(H);
  FreqWork W;
  {
    double2* q = reinterpret_cast<double2*>(sms);
    W.Z = q; q += 3 * H + 1;
    W.mu = q; q += 2 * H + 1;
    W.eta = q; q += H + 1;
    W.r = q; q += K + 1;
    W.al = q;
  }
  // shared phase: the record holds conj(B_n) in place of Z_n, so unit alpha
  // gives Mbar; the degeneracy scale comes from the bands' templates
  for (int q = lane; q < H; q += 64) W.al[q] = a.n_band ? make_double2(1.0, 0.0) : a.alpha[q];
  wave_sync();
  const double floor_mm = a.n_band ? a.mm_tau * a.lcs[0].mm_scale : mm_floor(W, H, a.mm_tau);
  // the record fields each lane needs (lane d <= K: r_d; e <= 2H: mu_e;
  // k < H: eta, Z_w; candidates c = lane + 64 s < D) are loaded one pair
  // ahead, so their latency overlaps the scoring of the current pair
  struct Fields { double2 r, mu, eta, zw; double cand[NSL]; };
  const int64_t n = list ? (int64_t)*list_n : np;
  auto item = [&](int64_t i) { return list ? list[i] : i; };
  auto fetch = [&](int64_t i) {
    Fields f;
    f.r = f.mu = f.eta = f.zw = make_double2(0.0, 0.0);
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) f.cand[sl] = 0.0;
    if (i < n) {
      const double* R = rec + item(i) * (int64_t)RL.stride;
      if (lane <= K) f.r = make_double2(R[RL.r + 2 * lane], R[RL.r + 2 * lane + 1]);
      if (lane <= 2 * H) f.mu = make_double2(R[RL.mu + 2 * lane], R[RL.mu + 2 * lane + 1]);
      if (lane < H) {
        f.eta = make_double2(R[RL.eta + 2 * lane], R[RL.eta + 2 * lane + 1]);
        f.zw = make_double2(R[RL.zw + 2 * lane], R[RL.zw + 2 * lane + 1]);
      }
#pragma unroll
      for (int sl = 0; sl < NSL; ++sl)
        if (lane + 64 * sl < D) f.cand[sl] = R[RL.cand + 64 * sl + lane];
    }
    return f;
  };
  Fields nxt = fetch(blockIdx.x);
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const Fields cur = nxt;
    nxt = fetch(i + gridDim.x);
    const int64_t w = item(i);
    const int64_t pidx = p0 + w;
    const double* Rr = rec + w * (int64_t)RL.stride;
    const int st = (int)Rr[RL.meta + M_STATUS];
    const int64_t lc = (int64_t)Rr[RL.meta + M_LC];
    const LcInfo& L = a.lcs[lc];
    if (st == ST_BAD_LC) {
      if (lane == 0) {
        a.power[pidx] = 0.0; a.phase[pidx] = 0.0; a.amp[pidx] = 0.0; a.offset[pidx] = 0.0;
        if (a.status) a.status[pidx] = ST_BAD_LC;
      }
      continue;
    }
    const double ref = Rr[RL.meta + M_REF];
    if (lane <= K) W.r[lane] = cur.r;
    if (lane <= 2 * H) W.mu[lane] = cur.mu;
    if (lane < H) {
      W.eta[lane + 1] = cur.eta;
      // the conjugated psi^k coefficient of Mbar, conj(alpha_k conj(Z_k))
      W.Z[lane + 1] = cconj(cmul(W.al[lane], cconj(cur.zw)));
    }
    if (lane == 0) W.eta[0] = make_double2(0.0, 0.0);
    wave_sync();
    double th[NSL];
    bool valid[NSL];
    Cand c[NSL];
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      th[sl] = 0.0;
      valid[sl] = false;
      if (st == ST_CONSTANT) {
        // P does not depend on the phase: score theta_2 = 0 (absolute)
        th[sl] = -kTwoPi * ref;
        valid[sl] = lane == 0 && sl == 0;
      } else if (lane + 64 * sl < D) {
        th[sl] = cur.cand[sl];
        valid[sl] = !isnan(th[sl]);
        if (!valid[sl]) th[sl] = 0.0;
      }
      c[sl] = eval_candidate(W, H, th[sl]);
    }
    double mml = valid[0] ? c[0].MM : -1.0;
    if (NSL > 1) mml = fmax(mml, valid[NSL - 1] ? c[NSL - 1].MM : -1.0);
    const double mmmax = wave_max(mml);
    int stout = st;
    if (mmmax <= floor_mm) stout = ST_DEGENERATE;
    // positive-amplitude variant: only candidates with theta_1 = YM/MM > 0
    const bool pos = (a.flags & kFlagPositiveAmp) != 0u;
    bool ok[NSL];
    bool any_ok = false;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      ok[sl] = valid[sl] && (c[sl].MM > floor_mm || stout == ST_DEGENERATE) && (!pos || c[sl].YM > 0.0);
      any_ok = any_ok || ok[sl];
    }
    const bool none = pos && stout != ST_DEGENERATE && __ballot(any_ok) == 0ull;
    Best b;
    int bslot = 0;
    if constexpr (NSL == 1) {
      b = select_best(c[0].P, th[0], wrap_2pi(th[0] + kTwoPi * ref), c[0].YM, ok[0], lane);
    } else {
      const double P2[2] = {c[0].P, c[NSL - 1].P}, ym2[2] = {c[0].YM, c[NSL - 1].YM};
      const double th2[2] = {th[0], th[NSL - 1]};
      const double ta2[2] = {wrap_2pi(th[0] + kTwoPi * ref), wrap_2pi(th[NSL - 1] + kTwoPi * ref)};
      const bool ok2[2] = {ok[0], ok[NSL - 1]};
      b = select_best2(P2, th2, ta2, ym2, ok2, bslot);
    }
    // Newton polish of the winner on R(theta) (Eq. theta2cond): a step is
    // kept only if it is small and P does not drop; a step below 1e-13 rad
    // changes P by O(1e-26) and ends the polish without re-scoring
    double best_th = b.th_rel;
    const Cand& cw = c[0];
    Cand cb = {__shfl(cw.P, b.lane), __shfl(cw.YM, b.lane), __shfl(cw.MM, b.lane), __shfl(cw.Mbar, b.lane)};
    if (NSL > 1 && bslot) {
      const Cand& cx = c[NSL - 1];
      cb = Cand{__shfl(cx.P, b.lane), __shfl(cx.YM, b.lane), __shfl(cx.MM, b.lane), __shfl(cx.Mbar, b.lane)};
    }
    // roots that Newton already converged (steps below 1e-12 rad, learned and
    // uniform solvers) are not polished: the polish step would be rounding noise
    const bool newton_root = a.newton_cands && Rr[RL.meta + M_FALLBACK] == 0.0;
    if (stout != ST_DEGENERATE && stout != ST_CONSTANT && !none && !newton_root) {
      for (int it = 0; it < 3; ++it) {
        double Rv, dR;
        eval_R(W, H, best_th, Rv, dR);
        if (!(dR != 0.0) || !isfinite(Rv / dR)) break;
        const double step = Rv / dR;
        if (fabs(step) > 1e-3 || fabs(step) < 1e-13) break;
        const double nt = best_th - step;
        const Cand nc = eval_candidate(W, H, nt);
        if (!(nc.P >= cb.P)) break;
        best_th = nt;
        cb = nc;
      }
    }
    if (lane == 0) {
      const double sq = sqrt(L.yy);
      double P = cb.P, amp = cb.MM > 0.0 ? cb.YM / cb.MM * sq : 0.0;
      double off = L.ybar - cb.Mbar * amp;
      double th_abs = wrap_2pi(best_th + kTwoPi * ref);
      if (stout == ST_DEGENERATE || none) { P = 0.0; amp = 0.0; off = L.ybar; th_abs = 0.0; }
      a.power[pidx] = P;
      a.phase[pidx] = th_abs;
      a.amp[pidx] = amp;
      a.offset[pidx] = off;
      const double fb = Rr[RL.meta + M_FALLBACK];
      const int fbits = fb >= 2.0 ? (ST_FALLBACK | ST_FALLBACK_QR) : (fb != 0.0 ? ST_FALLBACK : 0);
      if (a.status) a.status[pidx] = (uint8_t)(stout | fbits);
    }
    wave_sync();
  }
}


// Writes the deconvolved sums of every pair (3H complex per pair: Z_w(k j),
// k = 1..2H, then Z_y(k j), k = 1..H with the 1/sqrt(YY) normalisation undone).
// Maximum of a double over each 16-lane row, in every lane of the row.
__device__ __forceinline__ double row_max_d(double v) {
  v = fmax(v, dpp_d<0xB1>(v));    // quad_perm [1, 0, 3, 2]
  v = fmax(v, dpp_d<0x4E>(v));    // quad_perm [2, 3, 0, 1]
  v = fmax(v, dpp_d<0x141>(v));   // row_half_mirror
  v = fmax(v, dpp_d<0x140>(v));   // row_mirror
  return v;
}

// select_best within each 16-lane row over two candidates per lane (slot 0:
// candidate l, slot 1: candidate 16 + l of the row's frequency); the same
// rule, and the same winner, as select_best over the row's candidates in
// index order.  `slot` receives the winner's slot.
__device__ __forceinline__ Best select_best_row(const double (&P)[2], const double (&th_rel)[2],
                                                const double (&th_abs)[2], const double (&ym)[2],
                                                const bool (&valid)[2], int lane, int& slot) {
  const int row = lane >> 4;
  const double p0 = valid[0] ? P[0] : -1.0, p1 = valid[1] ? P[1] : -1.0;
  const double pmax = row_max_d(fmax(p0, p1));
  const double lo = pmax - 1e-12 * fmax(pmax, 1e-300);
  const bool n0 = valid[0] && p0 >= lo, n1 = valid[1] && p1 >= lo;
  const double k0 = n0 ? ((ym[0] > 0.0 ? 0.0 : 8.0) + th_abs[0]) : 1e30;
  const double k1 = n1 ? ((ym[1] > 0.0 ? 0.0 : 8.0) + th_abs[1]) : 1e30;
  const double kmin = -row_max_d(-fmin(k0, k1));
  const unsigned m0 = (unsigned)(__ballot(n0 && k0 == kmin) >> (16 * row)) & 0xffffu;
  const unsigned m1 = (unsigned)(__ballot(n1 && k1 == kmin) >> (16 * row)) & 0xffffu;
  slot = m0 ? 0 : (m1 ? 1 : 0);
  const unsigned m = m0 ? m0 : m1;
  Best b;
  b.lane = (m ? __ffs(m) - 1 : 0) + 16 * row;
  b.P = slot ? __shfl(p1, b.lane) : __shfl(p0, b.lane);
  b.th_rel = slot ? __shfl(th_rel[1], b.lane) : __shfl(th_rel[0], b.lane);
  b.th_abs = slot ? __shfl(th_abs[1], b.lane) : __shfl(th_abs[0], b.lane);
  b.amp_sign = slot ? __shfl(ym[1], b.lane) : __shfl(ym[0], b.lane);
  return b;
}

// Scoring of the first round's Newton-root pairs (M_FALLBACK = 0), four
// frequencies per wavefront, one per 16-lane row: the roots (at most 32 per
// frequency, its starts) are scored 16 at a time, and the candidates 16..31
// of a row take a second evaluation only when some row of the wavefront has
// more than 16 roots (a frequency has ~12 real roots at H = 10).  The
// candidates, tie rule and outputs of k_score, without the polish (the roots
// are Newton-converged).
//
// The record fields a row's lanes read (meta; mu_e, e = l, l + 16 <= 2H;
// eta_k and Z_w k, k = l < H; candidates l, l + 16) are loaded one iteration
// ahead, so that their latency overlaps the scoring of the current four pairs
// (2H + 1 <= 31 and H <= 15: two, one, one and two per lane cover them).
struct Score4Fetch {
  double st, fb, lc, ref, c0, c1;
  double2 mu0, mu1, eta, zw;
};

__device__ __forceinline__ void score4_fetch(const double* rec, const RecLayout& RL, int H, int ncand, int64_t np,
                                             int64_t w0, int row, int l, Score4Fetch& F) {
  const bool has = w0 + row < np;
  const double* Rr = rec + (has ? w0 + row : w0) * (int64_t)RL.stride;
  const double2 z = make_double2(0.0, 0.0);
  const double qnan = __longlong_as_double(0x7ff8000000000000ll);
  F.st = Rr[RL.meta + M_STATUS];
  F.fb = has ? Rr[RL.meta + M_FALLBACK] : 1.0;   // past the end: scored, never written
  F.lc = Rr[RL.meta + M_LC];
  F.ref = Rr[RL.meta + M_REF];
  const double2* mu = reinterpret_cast<const double2*>(Rr + RL.mu);
  F.mu0 = l <= 2 * H ? mu[l] : z;
  F.mu1 = l + 16 <= 2 * H ? mu[l + 16] : z;
  F.eta = l < H ? reinterpret_cast<const double2*>(Rr + RL.eta)[l] : z;
  F.zw = l < H ? reinterpret_cast<const double2*>(Rr + RL.zw)[l] : z;
  F.c0 = l < ncand ? Rr[RL.cand + l] : qnan;
  F.c1 = l + 16 < ncand ? Rr[RL.cand + l + 16] : qnan;
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_score4(SolveArgs a, const double* rec,
                                                                                       int64_t p0, int64_t np) {
  extern __shared__ double sms[];
  const int lane = wave_lane(), row = lane >> 4, l = lane & 15;
  const int H = a.H, K = 3 * H - 1, D = 2 * K;
  const RecLayout RL(H);
  FreqWork W;
  {
    double2* q = reinterpret_cast<double2*>(sms + row * (score_lds_bytes(H) / sizeof(double)));
    W.Z = q; q += 3 * H + 1;
    W.mu = q; q += 2 * H + 1;
    W.eta = q; q += H + 1;
    W.r = q; q += K + 1;
    W.al = q;
  }
  for (int q = l; q < H; q += 16) W.al[q] = a.n_band ? make_double2(1.0, 0.0) : a.alpha[q];
  wave_sync();
  const double floor_mm = a.n_band ? a.mm_tau * a.lcs[0].mm_scale : mm_floor(W, H, a.mm_tau);
  const bool pos = (a.flags & kFlagPositiveAmp) != 0u;
  const int ncand = D < 32 ? D : 32;   // the first round's starts per frequency
  const int64_t step = 4 * (int64_t)gridDim.x;
  Score4Fetch F;
  int64_t w0 = 4 * (int64_t)blockIdx.x;
  if (w0 < np) score4_fetch(rec, RL, H, ncand, np, w0, row, l, F);
  for (; w0 < np; w0 += step) {
    // this iteration's fields into LDS and registers, then the next
    // iteration's loads
    const int64_t pidx = p0 + (w0 + row < np ? w0 + row : w0);
    const int st = (int)F.st;
    const bool mine = F.fb == 0.0;
    const int64_t lc = (int64_t)F.lc;
    const double ref = F.ref;
    if (l <= 2 * H) W.mu[l] = F.mu0;
    if (l + 16 <= 2 * H) W.mu[l + 16] = F.mu1;
    if (l < H) {
      W.eta[l + 1] = F.eta;
      W.Z[l + 1] = cconj(cmul(W.al[l], cconj(F.zw)));
    }
    if (l == 0) W.eta[0] = make_double2(0.0, 0.0);
    double th[2] = {0.0, 0.0};
    bool valid[2] = {false, false};
    if (st == ST_CONSTANT) {
      th[0] = -kTwoPi * ref;
      valid[0] = l == 0;
    } else if (st != ST_BAD_LC) {
      th[0] = F.c0;
      th[1] = F.c1;
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        valid[sl] = !isnan(th[sl]);
        if (!valid[sl]) th[sl] = 0.0;
      }
    }
    if (w0 + step < np) score4_fetch(rec, RL, H, ncand, np, w0 + step, row, l, F);
    wave_sync();
    // (the evaluation reads mu, eta and Z: the Newton roots take no polish on R)
    const bool second = __ballot(valid[1]) != 0ull;   // wave-uniform
    Cand c[2];
    c[1] = Cand{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int sl = 0; sl < (second ? 2 : 1); ++sl) {
      const Cand t = eval_candidate(W, H, sl ? th[1] : th[0]);
      if (sl) c[1] = t; else c[0] = t;
    }
    const double mmmax = row_max_d(fmax(valid[0] ? c[0].MM : -1.0, valid[1] ? c[1].MM : -1.0));
    int stout = st;
    if (st != ST_BAD_LC && mmmax <= floor_mm) stout = ST_DEGENERATE;
    bool ok[2];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl)
      ok[sl] = valid[sl] && (c[sl].MM > floor_mm || stout == ST_DEGENERATE) && (!pos || c[sl].YM > 0.0);
    const unsigned okm = (unsigned)(__ballot(ok[0] || ok[1]) >> (16 * row)) & 0xffffu;
    const bool none = pos && stout != ST_DEGENERATE && okm == 0u;
    const double P2[2] = {c[0].P, c[1].P}, ym2[2] = {c[0].YM, c[1].YM};
    const double ta2[2] = {wrap_2pi(th[0] + kTwoPi * ref), wrap_2pi(th[1] + kTwoPi * ref)};
    int bslot;
    const Best b = select_best_row(P2, th, ta2, ym2, ok, lane, bslot);
    Cand cb = {__shfl(c[0].P, b.lane), __shfl(c[0].YM, b.lane), __shfl(c[0].MM, b.lane), __shfl(c[0].Mbar, b.lane)};
    if (bslot) cb = Cand{__shfl(c[1].P, b.lane), __shfl(c[1].YM, b.lane), __shfl(c[1].MM, b.lane), __shfl(c[1].Mbar, b.lane)};
    if (l == 0 && mine) {
      if (st == ST_BAD_LC) {
        a.power[pidx] = 0.0; a.phase[pidx] = 0.0; a.amp[pidx] = 0.0; a.offset[pidx] = 0.0;
        if (a.status) a.status[pidx] = ST_BAD_LC;
      } else {
        const LcInfo& L = a.lcs[lc];
        const double sq = sqrt(L.yy);
        double P = cb.P, amp = cb.MM > 0.0 ? cb.YM / cb.MM * sq : 0.0;
        double off = L.ybar - cb.Mbar * amp;
        double th_abs = wrap_2pi(b.th_rel + kTwoPi * ref);
        if (stout == ST_DEGENERATE || none) { P = 0.0; amp = 0.0; off = L.ybar; th_abs = 0.0; }
        a.power[pidx] = P;
        a.phase[pidx] = th_abs;
        a.amp[pidx] = amp;
        a.offset[pidx] = off;
        if (a.status) a.status[pidx] = (uint8_t)stout;
      }
    }
    wave_sync();
  }
}

template <typename R>
__global__ __launch_bounds__(64) void k_gather_sums(SolveArgs a, double* out) {
  const int lane = wave_lane();
  const int H = a.H;
  const typename Cplx<R>::T* grids = reinterpret_cast<const typename Cplx<R>::T*>(a.grids);
  for (int64_t pidx = blockIdx.x; pidx < a.total; pidx += gridDim.x) {
    const int64_t lc = pair_lc(a, pidx);
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

// chi^2_0 of each lightcurve of a chunk (Section 2.2): sum (y - ybar)^2 /
// sigma^2 = YY / w_inv with YY = sum w (y - ybar)^2, sum w = 1 (unit weights:
// w_inv = 1/N); 0 for a rejected lightcurve.
__global__ __launch_bounds__(256) void k_lc_chi2(const LcInfo* lcs, int64_t n_lc, double* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n_lc) out[i] = lcs[i].status == 0 ? lcs[i].yy / lcs[i].winv : 0.0;
}

// Multi-phase multi-band combination (Section 2.2, Eq.
// multibandmultiphase): power[j] = sum_k chi2[k] P_k[j] / sum_k chi2[k] over
// the band periodograms P_k = bp[k n_f + j]; 0 when every band was rejected.
__global__ __launch_bounds__(256) void k_mb_combine(const double* bp, int64_t n_band, int64_t n_f,
                                                    const double* chi2, double* power) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n_f) return;
  double num = 0.0, den = 0.0;
  for (int64_t k = 0; k < n_band; ++k) {
    num += chi2[k] * bp[k * n_f + j];
    den += chi2[k];
  }
  power[j] = den > 0.0 ? num / den : 0.0;
}

// Clears n counters (a kernel rather than a memset node, so that captured
// graphs replay it like any other launch).
__global__ __launch_bounds__(256) void k_zero_u32(unsigned* p, int64_t n, unsigned* p2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    p[i] = 0u;
    if (p2) p2[i] = 0u;
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

// ------------------------------------------------------------ launchers

template <int N>
static hipError_t launch_qr_n(double* rec, int stride, int64_t np, const int64_t* list,
                              const unsigned* list_count, SolveCounters* counters, unsigned* queue, int waves,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_qr<N>, dim3((unsigned)waves), dim3(64), qr_lds_bytes(N), st, rec, stride, np, list,
                     list_count, counters, queue);
  return hipGetLastError();
}

hipError_t launch_qr(int H, double* rec, int stride, int64_t np, const int64_t* list, const unsigned* list_count,
                     SolveCounters* counters, unsigned* queue, int waves, hipStream_t st) {
  switch (H) {
    case 1: return launch_qr_n<4>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 2: return launch_qr_n<10>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 3: return launch_qr_n<16>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 4: return launch_qr_n<22>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 5: return launch_qr_n<28>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 6: return launch_qr_n<34>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 7: return launch_qr_n<40>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 8: return launch_qr_n<46>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 9: return launch_qr_n<52>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 10: return launch_qr_n<58>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 11: return launch_qr_n<64>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 12: return launch_qr_n<70>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 13: return launch_qr_n<76>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 14: return launch_qr_n<82>(rec, stride, np, list, list_count, counters, queue, waves, st);
    case 15: return launch_qr_n<88>(rec, stride, np, list, list_count, counters, queue, waves, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_assemble(int precision, const SolveArgs& a, double* rec, int64_t p0, int64_t np, int waves,
                           hipStream_t st) {
  if (a.n_band == 0 && !a.sums_in && 6 * a.H - 2 < 64) {
    // two frequencies per wavefront, kAsmWaves wavefronts per workgroup
    const size_t lds2 = asm2_lds_bytes(a.H);
    const int64_t w2 = std::max<int64_t>(1, std::min<int64_t>(waves, (np + 1) / 2));
    const int g2 = (int)((w2 + kAsmWaves - 1) / kAsmWaves);
    if (precision == 1)
      hipLaunchKernelGGL(k_assemble2<double>, dim3((unsigned)g2), dim3(64 * kAsmWaves), lds2, st, a, rec, p0, np);
    else
      hipLaunchKernelGGL(k_assemble2<float>, dim3((unsigned)g2), dim3(64 * kAsmWaves), lds2, st, a, rec, p0, np);
    return hipGetLastError();
  }
  const size_t lds = asm_lds_bytes(a.H, a.n_band);
  if (precision == 1)
    hipLaunchKernelGGL(k_assemble<double>, dim3((unsigned)waves), dim3(64), lds, st, a, rec, p0, np);
  else
    hipLaunchKernelGGL(k_assemble<float>, dim3((unsigned)waves), dim3(64), lds, st, a, rec, p0, np);
  return hipGetLastError();
}

hipError_t launch_score(const SolveArgs& a, const double* rec, int64_t p0, int64_t np, int waves,
                        hipStream_t st, const int64_t* list, const unsigned* list_n) {
  if (6 * a.H - 2 > 64)
    hipLaunchKernelGGL(k_score<2>, dim3((unsigned)waves), dim3(64), score_lds_bytes(a.H), st, a, rec, p0, np, list,
                       list_n);
  else
    hipLaunchKernelGGL(k_score<1>, dim3((unsigned)waves), dim3(64), score_lds_bytes(a.H), st, a, rec, p0, np, list,
                       list_n);
  return hipGetLastError();
}

// Newton-candidate pairs four per wavefront (see k_score4); `done` (nullable):
// an event the launch itself records at the kernel's end.
hipError_t launch_score_newton(const SolveArgs& a, const double* rec, int64_t p0, int64_t np, int waves, hipStream_t st,
                         hipEvent_t done) {
  {
    // the first round's roots (at most 32 per frequency) in two rounds of a
    // 16-lane row: four frequencies per wavefront
    const int w4 = (int)std::max<int64_t>(1, std::min<int64_t>(waves, (np + 3) / 4));
    hipExtLaunchKernelGGL(k_score4, dim3((unsigned)w4), dim3(64), 4 * score_lds_bytes(a.H), st, nullptr, done, 0, a,
                          rec, p0, np);
    return hipGetLastError();
  }
}

hipError_t launch_gather_sums(int precision, const SolveArgs& a, double* out, int blocks, hipStream_t st) {
  if (precision == 1)
    hipLaunchKernelGGL(k_gather_sums<double>, dim3((unsigned)blocks), dim3(64), 0, st, a, out);
  else
    hipLaunchKernelGGL(k_gather_sums<float>, dim3((unsigned)blocks), dim3(64), 0, st, a, out);
  return hipGetLastError();
}

hipError_t launch_lc_chi2(const LcInfo* lcs, int64_t n_lc, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_lc_chi2, dim3((unsigned)((n_lc + 255) / 256)), dim3(256), 0, st, lcs, n_lc, out);
  return hipGetLastError();
}

hipError_t launch_mb_combine(const double* bp, int64_t n_band, int64_t n_f, const double* chi2, double* power,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_mb_combine, dim3((unsigned)((n_f + 255) / 256)), dim3(256), 0, st, bp, n_band, n_f, chi2,
                     power);
  return hipGetLastError();
}

// Clears p[0..n) and, when given, p2[0..n) in one launch.
hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t st, unsigned* p2) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, p2);
  return hipGetLastError();
}

hipError_t launch_export_stats(const LcInfo* lcs, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_export_stats, dim3(1), dim3(64), 0, st, lcs, out);
  return hipGetLastError();
}

}  // namespace ftp
