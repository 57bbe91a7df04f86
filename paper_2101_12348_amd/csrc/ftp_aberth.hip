// All roots of the Cayley polynomial f by the Aberth-Ehrlich simultaneous
// iteration (O. Aberth, Math. Comp. 27 (1973); L. W. Ehrlich, Comm. ACM 10
// (1967)), one root per lane of a wavefront.  A project addition to the
// method: the paper takes the roots of the phase polynomial (Eq. finalpoly)
// from a companion-matrix eigensolver; this kernel reaches the same root set
// by a different iteration and feeds the same candidate scoring.
//
// Used as the second tier of the learned solve (frequencies whose Newton
// roots the Sturm count did not confirm) and as a solver of its own over all
// frequencies.  Stopping rule: a lane stops when its correction is at the
// rounding level of |z| or when |f(z)| is within 4 D u of sum |f_k| |z|^k (the
// root is exact for a polynomial perturbed at rounding level, the backward
// error test of Bini and Fiorentino's MPSolve).  Frequencies whose roots do
// not all stop within kAberthMaxIt sweeps go to the companion-matrix solve.
//
// Candidates: each root x maps back to the phase
//   theta = phi0 + atan2(Re x, 1 - Im x) + atan2(Re x, 1 + Im x),
// the argument of psi = e^{i phi0} (1 + i x) / (1 - i x), i.e. the projection
// of psi onto the unit circle (Section 2, after Eq. finalpoly); a conjugate pair gives the same
// phase twice.
#include "ftp_solve_common.h"
#include "ftp_args.h"

namespace ftp {

constexpr int kAberthMaxIt = 60;

__host__ __device__ inline size_t aberth_lds_bytes(int H) {
  const int D = 6 * H - 2;
  return (size_t)((D + 2) + 2 * D) * sizeof(double);
}

__device__ __forceinline__ void awave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64) void k_aberth(AberthArgs A) {
  // the fallback tiers run beside the side stream's scoring: their waves
  // take issue priority over it on a shared SIMD (the tiers are few, latency-bound
  // waves on the step's critical path)
  __builtin_amdgcn_s_setprio(2);
  extern __shared__ double sab[];
  const int lane = threadIdx.x & 63;
  const int H = A.H, D = 6 * H - 2;
  const RecLayout RL(H);
  double* fc = sab;                                         // D + 1 coefficients
  double2* zs = reinterpret_cast<double2*>(sab + (D + 2));  // D roots (16-byte aligned: D even)
  const int64_t n = A.list ? (int64_t)(*A.count) : A.np;
  constexpr double u = 1.1102230246251565e-16;
  unsigned long long its_acc = 0, qr_acc = 0;
  for (int64_t i = first_item(A.queue, lane); i < n; i = next_item(A.queue, lane, i)) {
    const int64_t w = A.list ? A.list[i] : i;
    double* R = A.rec + w * (int64_t)RL.stride;
    if (!A.list) {
      const int st = (int)R[RL.meta + M_STATUS];
      if (st == ST_BAD_LC || st == ST_CONSTANT) continue;
    }
    if (A.flags & 1u) {
      if (lane == 0) {
        const unsigned slot = atomicAdd(A.qr_count, 1u);
        A.qr_list[slot] = w;
        R[RL.meta + M_FALLBACK] = A.mark;
        ++qr_acc;
      }
      continue;
    }
    double fmaxabs = 0.0;
    for (int c = lane; c <= D; c += 64) fmaxabs = fmax(fmaxabs, fabs(R[RL.f + c]));
    fmaxabs = wave_max(fmaxabs);
    const double fs = fmaxabs > 0.0 ? 1.0 / fmaxabs : 1.0;
    for (int c = lane; c <= D; c += 64) fc[c] = R[RL.f + c] * fs;
    awave_sync();
    const double f0 = fc[0], fD = fc[D];
    double rho = pow(fabs(f0 / fD), 1.0 / D);
    if (!(rho > 1e-8 && rho < 1e8)) rho = 1.0;
    const bool act = lane < D;
    // starting points: the real roots a Newton tier already found
    // (x = tan((theta - phi0) / 2)), the others on a circle of radius rho
    const int nw = A.list ? (int)R[RL.meta + M_WARM] : 0;
    const double phi0s = R[RL.meta + M_PHI0];
    double zr = 0.0, zi = 0.0;
    if (act && lane < nw) {
      zr = tan(0.5 * (R[RL.cand + lane] - phi0s));
      if (!isfinite(zr)) zr = 1e8;
    } else if (act) {
      double sn, cs;
      sincos(kTwoPi * (lane - nw + 0.25) / (D - nw), &sn, &cs);
      zr = rho * cs;
      zi = rho * sn;
    }
    bool done = !act;
    int it = 0;
    for (; it < kAberthMaxIt; ++it) {
      if (act) zs[lane] = make_double2(zr, zi);
      awave_sync();
      if (!done) {
        const double az = sqrt(zr * zr + zi * zi);
        double rr = 0.0, ri = 0.0;   // f'(z) / f(z)
        // one Horner loop for every lane (no divergent branches): inside the
        // unit circle f at x = z; outside, the reversed polynomial
        // g(y) = y^D f(1/y) at x = y = 1/z, with f'/f = y (D - y g'/g)
        const bool inside = az <= 1.0;
        double xr = zr, xi = zi, ax = az;
        if (!inside) {
          const double iz2 = 1.0 / (az * az);
          xr = zr * iz2;
          xi = -zi * iz2;
          ax = 1.0 / az;
        }
        const int c0 = inside ? D : 0, cs = inside ? -1 : 1;   // coefficient of x^D, then step
        double pr = fc[c0], pi = 0.0, dr = 0.0, di = 0.0, ab = fabs(fc[c0]);
        for (int k = 1; k <= D; ++k) {
          const double c = fc[c0 + cs * k];
          const double tr = dr * xr - di * xi + pr;
          di = dr * xi + di * xr + pi;
          dr = tr;
          const double qr = pr * xr - pi * xi + c;
          pi = pr * xi + pi * xr;
          pr = qr;
          ab = ab * ax + fabs(c);
        }
        const double pm2 = pr * pr + pi * pi;
        const bool exact = !(sqrt(pm2) > 4.0 * D * u * ab);
        if (!exact) {
          const double inv = 1.0 / pm2;
          const double qr = (dr * pr + di * pi) * inv, qi = (di * pr - dr * pi) * inv;   // p'/p at x
          if (inside) {
            rr = qr;
            ri = qi;
          } else {
            const double sr = D - (xr * qr - xi * qi), si = -(xr * qi + xi * qr);       // D - y g'/g
            rr = xr * sr - xi * si;
            ri = xr * si + xi * sr;
          }
        }
        if (exact) {
          done = true;
        } else {
          // sum_{j != lane} 1 / (z - z_j): the j = lane term is 1/0 -> skipped
          // by a select, so the loop body has no branch and unrolls
          double sr = 0.0, si = 0.0;
#pragma unroll 4
          for (int j = 0; j < D; ++j) {
            const double2 zj = zs[j];
            const double er = zr - zj.x, ei = zi - zj.y;
            const double inv = j == lane ? 0.0 : fast_rcp_d(er * er + ei * ei);
            sr += er * inv;
            si -= ei * inv;
          }
          const double br = rr - sr, bi = ri - si;
          const double inv = fast_rcp_d(br * br + bi * bi);
          const double cr = br * inv, ci = -bi * inv;   // correction 1 / (f'/f - S)
          if (isfinite(cr) && isfinite(ci)) {
            zr -= cr;
            zi -= ci;
            if (sqrt(cr * cr + ci * ci) <= 4.0 * u * sqrt(zr * zr + zi * zi)) done = true;
          } else {
            done = true;   // coincident estimates: leave to the verdict below
          }
        }
      }
      awave_sync();
      if (__ballot(!done) == 0ull) break;
    }
    // verdict: every lane stopped with a finite root, and the roots add up to
    // -f_{D-1} / f_D (Vieta), which two estimates stuck on one root would break
    const bool finite = !act || (isfinite(zr) && isfinite(zi));
    double sx = act ? zr : 0.0, sy = act ? zi : 0.0, sa = act ? sqrt(zr * zr + zi * zi) : 0.0;
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sa = wave_sum(sa);
    const double ex = sx + fc[D - 1] / fD;
    const bool vieta = sqrt(ex * ex + sy * sy) <= 1e-8 * (sa + fabs(fc[D - 1] / fD)) + 1e-12;
    const bool ok = it < kAberthMaxIt && __ballot(!finite) == 0ull && vieta;
    its_acc += (unsigned long long)(it < kAberthMaxIt ? it + 1 : it);
    if (ok) {
      const double phi0 = R[RL.meta + M_PHI0];
      double* cand = R + RL.cand;
      if (act) cand[lane] = phi0 + atan2(zr, 1.0 - zi) + atan2(zr, 1.0 + zi);
    } else if (lane == 0) {
      const unsigned slot = atomicAdd(A.qr_count, 1u);
      A.qr_list[slot] = w;
      R[RL.meta + M_FALLBACK] = A.mark;
      ++qr_acc;
    }
    awave_sync();
  }
  if (lane == 0 && A.counters) {
    if (its_acc) atomicAdd(&counter_slot(A.counters)->aberth_iters, its_acc);
    if (qr_acc) atomicAdd(&counter_slot(A.counters)->fallback_qr, qr_acc);
  }
}

// The same iteration for the fallback tier (a list of a few frequencies, D <
// 64) with kAbW wavefronts per frequency: the GPU is otherwise idle while the
// tier runs, and its time is the slowest frequency's sweeps, so each sweep is
// split.  Wave w evaluates the powers c0_w .. c1_w - 1 of the lane's
// polynomial (a_c = f_c inside the unit circle, f_{D-c} for the reversed one
// outside) by Horner and scales them by x^c0_w (V = x^c0 Q, V' = c0 x^(c0-1) Q +
// x^c0 Q'), and sums 1 / (z - z_j) over its quarter of the roots; the
// partials meet in LDS and every wave adds them in the same order, so that
// all waves hold the same roots.  Two barriers per sweep.
constexpr int kAbW = 4;

__host__ __device__ inline size_t aberth_split_lds_bytes(int H) {
  const int D = 6 * H - 2;
  return (size_t)((D + 2) + 2 * D + kAbW * 7 * 64) * sizeof(double);
}

__global__ __launch_bounds__(64 * kAbW) void k_aberth_split(AberthArgs A) {
  // the fallback tiers run beside the side stream's scoring: their waves
  // take issue priority over it on a shared SIMD (the tiers are few, latency-bound
  // waves on the step's critical path)
  __builtin_amdgcn_s_setprio(2);
  extern __shared__ double sab[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int H = A.H, D = 6 * H - 2;
  const RecLayout RL(H);
  double* fc = sab;                                          // D + 1 coefficients
  double2* zs = reinterpret_cast<double2*>(sab + (D + 2));   // D roots (16-byte aligned: D even)
  double* part = sab + (D + 2) + 2 * D;                      // [wave][7][64] partials
  const int64_t n = (int64_t)(*A.count);
  constexpr double u = 1.1102230246251565e-16;
  unsigned long long its_acc = 0, qr_acc = 0;
  const int cseg = (D + 1 + kAbW - 1) / kAbW, jseg = (D + kAbW - 1) / kAbW;
  const int cw0 = min(wv * cseg, D + 1), cw1 = min(cw0 + cseg, D + 1);
  const int jw0 = min(wv * jseg, D), jw1 = min(jw0 + jseg, D);
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t w = A.list[i];
    double* R = A.rec + w * (int64_t)RL.stride;
    if (A.flags & 1u) {
      if (tid == 0) {
        const unsigned slot = atomicAdd(A.qr_count, 1u);
        A.qr_list[slot] = w;
        R[RL.meta + M_FALLBACK] = A.mark;
        ++qr_acc;
      }
      continue;
    }
    // every wave forms the same scale, starting points and verdict
    const double fv = lane <= D ? R[RL.f + lane] : 0.0;
    const double fmaxabs = wave_max(fabs(fv));
    const double fs = fmaxabs > 0.0 ? 1.0 / fmaxabs : 1.0;
    if (wv == 0 && lane <= D) fc[lane] = fv * fs;
    __syncthreads();
    const double f0 = fc[0], fD = fc[D];
    double rho = pow(fabs(f0 / fD), 1.0 / D);
    if (!(rho > 1e-8 && rho < 1e8)) rho = 1.0;
    const bool act = lane < D;
    const int nw = (int)R[RL.meta + M_WARM];
    const double phi0s = R[RL.meta + M_PHI0];
    double zr = 0.0, zi = 0.0;
    if (act && lane < nw) {
      zr = tan(0.5 * (R[RL.cand + lane] - phi0s));
      if (!isfinite(zr)) zr = 1e8;
    } else if (act) {
      double sn, cs;
      sincos(kTwoPi * (lane - nw + 0.25) / (D - nw), &sn, &cs);
      zr = rho * cs;
      zi = rho * sn;
    }
    bool done = !act;
    int it = 0;
    for (; it < kAberthMaxIt; ++it) {
      if (wv == 0 && act) zs[lane] = make_double2(zr, zi);
      __syncthreads();
      const double az = sqrt(zr * zr + zi * zi);
      const bool inside = az <= 1.0;
      double xr = zr, xi = zi, ax = az;
      if (!inside) {
        const double iz2 = 1.0 / (az * az);
        xr = zr * iz2;
        xi = -zi * iz2;
        ax = 1.0 / az;
      }
      {
        // this wave's powers: Q = sum_{c=cw0}^{cw1-1} a_c x^(c - cw0) and Q'
        const int cb = inside ? 0 : D, cs = inside ? 1 : -1;   // a_c = fc[cb + cs c]
        double pr = 0.0, pi = 0.0, dr = 0.0, di = 0.0, ab = 0.0;
        for (int c = cw1 - 1; c >= cw0; --c) {
          const double cc = fc[cb + cs * c];
          const double tr = dr * xr - di * xi + pr;
          di = dr * xi + di * xr + pi;
          dr = tr;
          const double qr = pr * xr - pi * xi + cc;
          pi = pr * xi + pi * xr;
          pr = qr;
          ab = ab * ax + fabs(cc);
        }
        // x^(cw0 - 1) by repeated squaring (x^0 for cw0 = 0), then x^cw0
        double2 pm = make_double2(1.0, 0.0), bsq = make_double2(xr, xi);
        double am = 1.0, absq = ax;
        for (int e = cw0 > 0 ? cw0 - 1 : 0; e; e >>= 1) {
          if (e & 1) {
            pm = cmul(pm, bsq);
            am *= absq;
          }
          bsq = cmul(bsq, bsq);
          absq *= absq;
        }
        const double2 px = cw0 > 0 ? cmul(pm, make_double2(xr, xi)) : pm;
        const double apx = cw0 > 0 ? am * ax : 1.0;
        const double2 q = make_double2(pr, pi), dq = make_double2(dr, di);
        const double2 v = cmul(px, q);
        const double2 vd = cadd(cscale(cmul(pm, q), (double)cw0), cmul(px, dq));
        // this wave's roots: sum 1 / (z - z_j), j = jw0 .. jw1 - 1 (j = lane skipped)
        double sr = 0.0, si = 0.0;
        for (int j = jw0; j < jw1; ++j) {
          const double2 zj = zs[j];
          const double er = zr - zj.x, ei = zi - zj.y;
          const double inv = j == lane ? 0.0 : fast_rcp_d(er * er + ei * ei);
          sr += er * inv;
          si -= ei * inv;
        }
        double* pw = part + wv * 7 * 64 + lane;
        pw[0] = v.x;
        pw[64] = v.y;
        pw[128] = vd.x;
        pw[192] = vd.y;
        pw[256] = sr;
        pw[320] = si;
        pw[384] = apx * ab;
      }
      __syncthreads();
      if (!done) {
        double pr = 0.0, pi = 0.0, dr = 0.0, di = 0.0, sr = 0.0, si = 0.0, ab = 0.0;
        for (int q = 0; q < kAbW; ++q) {
          const double* pq = part + q * 7 * 64 + lane;
          pr += pq[0];
          pi += pq[64];
          dr += pq[128];
          di += pq[192];
          sr += pq[256];
          si += pq[320];
          ab += pq[384];
        }
        const double pm2 = pr * pr + pi * pi;
        const bool exact = !(sqrt(pm2) > 4.0 * D * u * ab);
        if (exact) {
          done = true;
        } else {
          const double inv = 1.0 / pm2;
          const double qr = (dr * pr + di * pi) * inv, qi = (di * pr - dr * pi) * inv;   // q'/q at x
          double rr = qr, ri = qi;
          if (!inside) {
            const double s2r = D - (xr * qr - xi * qi), s2i = -(xr * qi + xi * qr);      // D - y g'/g
            rr = xr * s2r - xi * s2i;
            ri = xr * s2i + xi * s2r;
          }
          const double br = rr - sr, bi = ri - si;
          const double inv2 = fast_rcp_d(br * br + bi * bi);
          const double cr = br * inv2, ci = -bi * inv2;   // correction 1 / (f'/f - S)
          if (isfinite(cr) && isfinite(ci)) {
            zr -= cr;
            zi -= ci;
            if (sqrt(cr * cr + ci * ci) <= 4.0 * u * sqrt(zr * zr + zi * zi)) done = true;
          } else {
            done = true;   // coincident estimates: leave to the verdict below
          }
        }
      }
      if (__ballot(!done) == 0ull) break;   // the same in every wave
    }
    const bool finite = !act || (isfinite(zr) && isfinite(zi));
    double sx = act ? zr : 0.0, sy = act ? zi : 0.0, sa = act ? sqrt(zr * zr + zi * zi) : 0.0;
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sa = wave_sum(sa);
    const double ex = sx + fc[D - 1] / fD;
    const bool vieta = sqrt(ex * ex + sy * sy) <= 1e-8 * (sa + fabs(fc[D - 1] / fD)) + 1e-12;
    const bool ok = it < kAberthMaxIt && __ballot(!finite) == 0ull && vieta;
    if (wv == 0) {
      its_acc += (unsigned long long)(it < kAberthMaxIt ? it + 1 : it);
      if (ok) {
        const double phi0 = R[RL.meta + M_PHI0];
        if (act) R[RL.cand + lane] = phi0 + atan2(zr, 1.0 - zi) + atan2(zr, 1.0 + zi);
      } else if (lane == 0) {
        const unsigned slot = atomicAdd(A.qr_count, 1u);
        A.qr_list[slot] = w;
        R[RL.meta + M_FALLBACK] = A.mark;
        ++qr_acc;
      }
    }
    __syncthreads();   // LDS reused by the next frequency
  }
  if (tid == 0 && A.counters) {
    if (its_acc) atomicAdd(&counter_slot(A.counters)->aberth_iters, its_acc);
    if (qr_acc) atomicAdd(&counter_slot(A.counters)->fallback_qr, qr_acc);
  }
}

hipError_t launch_aberth(const AberthArgs& A, int waves, hipStream_t st) {
  if (6 * A.H - 2 > 64) {
    // degree above 64 (one root per lane does not fit): the tier hands its
    // list to the companion solve (the Aberth solver is refused at plan
    // creation for such H)
    AberthArgs F = A;
    F.flags |= 1u;
    hipLaunchKernelGGL(k_aberth, dim3((unsigned)waves), dim3(64), 0, st, F);
    return hipGetLastError();
  }
  if (A.list && 6 * A.H - 2 < 64) {
    // fallback tier: kAbW wavefronts per frequency, grid-strided over the list
    const int wg = waves / kAbW > 1 ? waves / kAbW : 1;
    hipLaunchKernelGGL(k_aberth_split, dim3((unsigned)wg), dim3(64 * kAbW), aberth_split_lds_bytes(A.H), st, A);
  } else {
    hipLaunchKernelGGL(k_aberth, dim3((unsigned)waves), dim3(64), aberth_lds_bytes(A.H), st, A);
  }
  return hipGetLastError();
}

}  // namespace ftp
