// Learned root proposal (a project addition to the method): Newton on the
// real phase polynomial from network seeds, verified by a Sturm count.
//
// For each frequency (one wavefront):
//   * the number of distinct real roots of R is counted with a Sturm sequence
//     of the Cayley polynomial f(x) (theta = phi0 + 2 atan x) over the whole
//     real line;
//   * if the count is well determined, 2H network seeds plus evenly spaced
//     starts (only evenly spaced starts for the ablation without network) are
//     refined by FP64 Newton on R(theta) = 2 MM dYM/dtheta - YM dMM/dtheta
//     (Eq. theta2cond written as R(theta) = i e^{-i K theta} p(e^{i theta})),
//     each step evaluated on the Cayley polynomial f with the iterate kept as
//     tan((theta - phi0) / 2) or its reciprocal (newton_u_step); converged
//     roots closer than 1e-8 rad are merged, one root per pass, after every
//     iteration from the fourth, and Newton stops once the merged roots reach
//     the count;
//   * if they do, the Newton roots are the candidate set; otherwise the
//     frequency goes to the Aberth iteration (then, if that does not
//     converge, to the companion-matrix solve) through device work lists.
// For H <= 10 a wavefront takes four frequencies (k_newton_sturm4): their
// Sturm sequences run one per 16-lane row with four coefficients per lane in
// registers, and Newton runs on two of them at a time (32 starts each, at
// most D).  For H = 11 a wavefront takes one (k_newton_sturm, 4H starts),
// its Sturm sequence one coefficient per lane (the degree-64 coefficient
// carried as a scalar; see sturm_begin).
#include <hip/hip_ext.h>
#include "ftp_solve_common.h"
#include "ftp_args.h"

namespace ftp {

__device__ __forceinline__ void lwave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double lrdlane(double v, int src) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), src);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

__device__ __forceinline__ int hiword(double x) {
  return (int)((unsigned long long)__double_as_longlong(x) >> 32);
}
__device__ __forceinline__ double from_hiword(int h) {
  return __longlong_as_double((long long)((unsigned long long)(unsigned)h << 32));
}

// Thresholds of the Sturm test, applied to high words of positive doubles: a
// difference of high words is 2^20 log2 of the ratio to within 0.09 (the
// mantissa enters linearly), so "ratio above 1e-12" reads hi(x) - hi(y) >
// hi(1) - hi(1e-12), to within 7% of the bound.  hi(NaN) and hi(inf) are at
// least 0x7ff00000.
constexpr int kHi1 = 0x3ff00000;
constexpr int kHiT12 = kHi1 - 0x3d719799;   // hi(1) - hi(1e-12)
constexpr int kHiT13 = kHi1 - 0x3d3c25c2;   // hi(1) - hi(1e-13)

// Maximum of an int over the wavefront (row stages, then row_bcast:15 and
// row_bcast:31 into lane 63).
__device__ __forceinline__ int wave_max_int(int h) {
  h = max(h, dpp_i<0xB1, 0xf>(h));
  h = max(h, dpp_i<0x4E, 0xf>(h));
  h = max(h, dpp_i<0x141, 0xf>(h));
  h = max(h, dpp_i<0x140, 0xf>(h));
  h = max(h, dpp_i<0x142, 0xa>(h));
  h = max(h, dpp_i<0x143, 0xc>(h));
  return __builtin_amdgcn_readlane(h, 63);
}

// The test of one Sturm step on high words: hr = hi(max |t|) of the
// remainder, hl = hi(|leading coefficient of t|), hM = hi of the larger of
// the two members' largest coefficient magnitudes.  The remainder must not
// vanish against the members (max |t| above 1e-12 of theirs: else a gcd of
// positive degree, repeated or nearly repeated roots) nor lose its leading
// term to cancellation (above 1e-13 of max |t|), and must be finite.
__device__ __forceinline__ bool sturm_step_ok(int hr, int hl, int hM) {
  return (hr < 0x7ff00000) & (hr - hM > -kHiT12) & (hl - hr > -kHiT13);
}
// hi(max |P_q|) of the scaled member P_q = -t / |lead|: hr - hl + hi(1)
// (bounded so that a failed chain's value stays an int)
__device__ __forceinline__ int sturm_member_hi(int hr, int hl) { return min(hr - hl, 0x40000000) + kHi1; }

// Sturm sequence of a degree-D polynomial g over the whole real line, D + 1
// <= 64, in registers: P_0 = g, P_1 = g', P_q = -rem(P_{q-2}, P_{q-1}), lane c
// holding coefficient c (the shift by one power of x is a DPP lane shift).
// Each member is scaled by the reciprocal of its leading coefficient's
// magnitude (P_0 and P_1 with their leading lane set to +-1): a positive scale
// leaves the signs, and so the count, unchanged, and the quotient of each
// division is taken as al bl x + (next coefficient) bl with al, bl = +-1 and no
// division (a member's leading coefficient is +-1 to within the reciprocal's
// few ulp, which perturbs the quotient by as much: the size of the rounding
// already present).  Every member of a generic sequence has degree D - q, so
// its signs at +inf and -inf are those of its leading coefficient (times
// (-1)^(D - q) at -inf), and the count V(-inf) - V(+inf) accumulates as the
// members are formed; consecutive members differ in degree by one, so at -inf
// a sign change occurs exactly where none occurs at +inf, and with V(+inf) =
// vp over the D transitions of a full chain the count is D - 2 vp.  Each step
// is tested (sturm_step_ok); a chain that fails is not trusted.
struct SturmChain {
  double A, B, al, bl;  // the last two members and their leading coefficients (+-1)
  int hMA, hMB;         // hi(max |coefficient|) of A and B
  int sp;               // last member positive at +inf (0 / 1)
  int vp;               // sign changes at +inf so far
  bool ok;
};

// gv: coefficient `lane` of g (lanes 0..min(D, 63)); gtop = g[D].  For D = 64
// the top coefficient has no lane: it is carried as the scalar leading
// coefficient only, which is all the chain needs of it (the first remainder
// cancels it exactly and the shifted derivative reaches lane 63 at most).
__device__ __forceinline__ SturmChain sturm_begin(double gv, double gtop, int D, int lane) {
  SturmChain c;
  const double gnext = lane_shl1(gv);   // g[lane + 1], taken with every lane active
  const double g1 = lane == 63 ? gtop : gnext;
  const double dv = lane < D ? (lane + 1) * g1 : 0.0;
  const double ag = fabs(gtop), sgn = gtop > 0.0 ? 1.0 : -1.0;
  const double sa = fast_rcp_d(ag + 1e-300), sb = fast_rcp_d(D * ag + 1e-300);
  c.ok = ag > 0.0 && ag < INFINITY;
  c.A = lane == D ? sgn : gv * sa;
  c.B = lane == D - 1 ? sgn : dv * sb;
  c.al = sgn;
  c.bl = sgn;
  c.hMA = max(wave_max_int(hiword(c.A) & 0x7fffffff), kHi1);   // the top of A is +-1 (no lane at D = 64)
  c.hMB = wave_max_int(hiword(c.B) & 0x7fffffff);
  c.vp = 0;
  c.sp = gtop > 0.0 ? 1 : 0;
  return c;
}

// Member q (2 <= q <= D) from the last two (every lane holds one chain).
// Branch-free, so that two chains stepped side by side interleave.
__device__ __forceinline__ void sturm_step(SturmChain& c, int D, int q, int lane) {
  const int db = D - q + 1;
  double t = c.A - (c.al * c.bl) * lane_shr1(c.B);
  const double q0 = lrdlane(t, db) * c.bl;
  t = lane < db ? t - q0 * c.B : 0.0;
  const double lead = lrdlane(t, db - 1);
  const int hl = hiword(lead), hla = hl & 0x7fffffff;
  const int hr = wave_max_int(hiword(t) & 0x7fffffff);
  c.ok = c.ok && sturm_step_ok(hr, hla, max(c.hMA, c.hMB));
  // P_q = -t / |lead|: positive at +inf when lead < 0 (sign bit of hl)
  const int tp = (int)((unsigned)hl >> 31);
  c.vp += tp ^ c.sp;
  c.sp = tp;
  const double s = fast_rcp_d(fabs(lead) + 1e-300);
  c.A = c.B;
  c.al = c.bl;
  c.hMA = c.hMB;
  c.B = -t * s;
  c.bl = from_hiword((hl & 0x80000000) ^ 0xbff00000);   // -sign(lead)
  c.hMB = sturm_member_hi(hr, hla);
}

// Distinct real roots of g (coefficient `gv` in lane c, gtop = g[D] != 0,
// D <= 64), or -1; `raw` receives the count whether or not the chain passed
// its tests (a diagnostic).
__device__ int sturm_count_line_reg(double gv, double gtop, int D, int lane, int& raw) {
  SturmChain c = sturm_begin(gv, gtop, D, lane);
  for (int q = 2; q <= D; ++q) sturm_step(c, D, q, lane);
  raw = D - 2 * c.vp;
  return c.ok ? raw : -1;
}

// ---- double-double arithmetic (value hi + lo, |lo| <= ulp(hi) / 2): the
// error-free transformations of Knuth (TAOCP vol. 2, two-sum) and Dekker
// (1971, the product, here through the fused multiply-add).  Contraction of
// a product into a later sum is off in these helpers: the error terms assume
// each operation rounded on its own (a fused p + e in the product's
// normalisation drops the double-double precision to double's).
struct dd { double hi, lo; };
__device__ __forceinline__ dd dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b, bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd dd_quick(double a, double b) {   // |a| >= |b|
#pragma clang fp contract(off)
  const double s = a + b;
  return dd{s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
  dd s = dd_two_sum(x.hi, y.hi);
  const dd t = dd_two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = dd_quick(s.hi, s.lo);
  s.lo += t.lo;
  return dd_quick(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd x) { return dd{-x.hi, -x.lo}; }
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
#pragma clang fp contract(off)
  const double p = x.hi * y.hi;
  double e = fma(x.hi, y.hi, -p);
  e = fma(x.hi, y.lo, fma(x.lo, y.hi, e));
  return dd_quick(p, e);
}
__device__ __forceinline__ dd dd_div(dd x, dd y) {
#pragma clang fp contract(off)
  // two quotient digits: q1 = x / y in double, q2 from the remainder
  const double q1 = x.hi / y.hi;
  const dd r = dd_add(x, dd_neg(dd_mul(dd{q1, 0.0}, y)));
  const double q2 = r.hi / y.hi;
  return dd_quick(q1, q2);
}
__device__ __forceinline__ dd dd_ldexp(dd x, int e) { return dd{ldexp(x.hi, e), ldexp(x.lo, e)}; }
__device__ __forceinline__ dd dd_lane(dd v, int src) { return dd{lrdlane(v.hi, src), lrdlane(v.lo, src)}; }
// v from lane - 1 (lane 0: 0), both parts
__device__ __forceinline__ dd dd_shr1(dd v) { return dd{lane_shr1(v.hi), lane_shr1(v.lo)}; }

// largest |v| over the wavefront, from the doubles' high words (within a
// factor 1 + 2^-20: enough for the chain's tests)
__device__ __forceinline__ double wave_max_abs(double v) {
  return from_hiword(wave_max_int(hiword(v) & 0x7fffffff));
}

// Distinct real roots of g for 64 < D <= 127 in double-double, or -1
// (`raw`: the count regardless of the tests).  Coefficient c = lane + 64 s of
// a member in register s.  Each remainder is the exact-arithmetic step
// (quotient q1 x + q0 from the two leading coefficients, by double-double
// division) and each member is scaled by a power of two that brings its
// leading coefficient into [1, 2) (exact).  The chain is trusted when every
// remainder's largest coefficient exceeds 1e-24 of the larger of its two
// members' and its leading coefficient 1e-24 of its largest, all finite: in
// double precision the spread of the Cayley polynomial's coefficients at
// these degrees (1e-15 .. 1e-19) defeats the 1e-13 test of the other chains,
// while 106 bits leave room (a 106-bit emulation of this chain trusted and
// matched the exact count on every polynomial tried at H = 12..15, also where
// a double-precision chain with a relaxed test was wrong).  All lanes active.
__device__ int sturm_count_dd(double g0, double g1, int D, int lane, int& raw) {
#pragma clang fp contract(off)
  const int c0 = lane, c1 = lane + 64;
  // g and g' (exact in double-double: (c + 1) g_{c+1} is one product)
  const double n0 = lane_shl1(g0), n1 = lane_shl1(g1);
  const double g64 = lrdlane(g1, 0);
  const double u0 = lane == 63 ? g64 : n0;
  dd A[2], B[2];
  A[0] = dd{g0, 0.0};
  A[1] = dd{g1, 0.0};
  {
    const double p0 = (double)(c0 + 1) * u0, p1 = (double)(c1 + 1) * n1;
    B[0] = c0 < D ? dd{p0, fma((double)(c0 + 1), u0, -p0)} : dd{0.0, 0.0};
    B[1] = c1 < D ? dd{p1, fma((double)(c1 + 1), n1, -p1)} : dd{0.0, 0.0};
  }
  // scale both to leading coefficients in [1, 2) in magnitude
  auto lead_of = [&](const dd (&X)[2], int deg) { return deg >= 64 ? dd_lane(X[1], deg - 64) : dd_lane(X[0], deg); };
  int e;
  {
    dd la = lead_of(A, D);
    frexp(la.hi, &e);
    A[0] = dd_ldexp(A[0], 1 - e);
    A[1] = dd_ldexp(A[1], 1 - e);
    dd lb = lead_of(B, D - 1);
    frexp(lb.hi, &e);
    B[0] = dd_ldexp(B[0], 1 - e);
    B[1] = dd_ldexp(B[1], 1 - e);
  }
  bool ok = lead_of(A, D).hi != 0.0 && isfinite(lead_of(A, D).hi) && lead_of(B, D - 1).hi != 0.0;
  double mA = wave_max_abs(fmax(fabs(A[0].hi), fabs(A[1].hi)));
  double mB = wave_max_abs(fmax(fabs(B[0].hi), fabs(B[1].hi)));
  int sp = lead_of(A, D).hi > 0.0 ? 1 : 0;
  int vp = 0;
  {
    const int tb = lead_of(B, D - 1).hi > 0.0 ? 1 : 0;
    vp += tb ^ sp;
    sp = tb;
  }
  for (int db = D - 1; db >= 1; --db) {   // B has degree db, A degree db + 1
    const bool two = db + 1 >= 64;         // (wave-uniform)
    const dd at = lead_of(A, db + 1), bt = lead_of(B, db);
    const dd q1 = dd_div(at, bt);
    // t = A - q1 x B (the coefficient db + 1 cancels)
    dd sh0 = dd_shr1(B[0]), sh1 = dd_shr1(B[1]);
    const dd b63 = dd_lane(B[0], 63);
    if (lane == 0) sh1 = b63;
    dd t0 = dd_add(A[0], dd_neg(dd_mul(q1, sh0)));
    dd t1 = two ? dd_add(A[1], dd_neg(dd_mul(q1, sh1))) : dd{0.0, 0.0};
    const dd ct = db >= 64 ? dd_lane(t1, db - 64) : dd_lane(t0, db);
    const dd q0 = dd_div(ct, bt);
    // rem = -(t - q0 B): coefficients below db
    t0 = c0 < db ? dd_neg(dd_add(t0, dd_neg(dd_mul(q0, B[0])))) : dd{0.0, 0.0};
    t1 = (two && c1 < db) ? dd_neg(dd_add(t1, dd_neg(dd_mul(q0, B[1])))) : dd{0.0, 0.0};
    const dd lead = db - 1 >= 64 ? dd_lane(t1, db - 65) : dd_lane(t0, db - 1);
    const double mr = wave_max_abs(fmax(fabs(t0.hi), fabs(t1.hi)));
    ok = ok && isfinite(mr) && mr > 1e-24 * fmax(mA, mB) && fabs(lead.hi) > 1e-24 * mr;
    const int tp = lead.hi > 0.0 ? 1 : 0;
    vp += tp ^ sp;
    sp = tp;
    frexp(lead.hi, &e);
    if (!(lead.hi != 0.0 && isfinite(lead.hi))) e = 0;
    A[0] = B[0];
    A[1] = B[1];
    B[0] = dd_ldexp(t0, 1 - e);
    B[1] = dd_ldexp(t1, 1 - e);
    mA = mB;
    mB = ldexp(mr, 1 - e);
  }
  raw = D - 2 * vp;
  return ok ? raw : -1;
}

// v from lane addr / 4 (ds_bpermute, all lanes active)
__device__ __forceinline__ double bperm_d(int addr, double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(u & 0xffffffffull));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Four Sturm chains per wavefront, one per 16-lane row.  Lane 16 c + l holds
// coefficients 16 r + l (r = 0..3) of chain c's members in registers, so a
// member of up to 64 coefficients needs no LDS and every instruction of a
// step serves four chains: the shift by one power of x is a row rotation
// (DPP row_ror:1, lane 0 taking lane 15 of the register below), the two
// coefficients a step needs from its own chain (the quotient's and the new
// leading coefficient) come by ds_bpermute from the row's lane, and the
// largest coefficient by a row all-reduction.  Per coefficient the arithmetic
// is that of sturm_begin / sturm_step (scaled members with leading
// coefficient +-1, quotients without division, the same step test on high
// words), and a step only touches the registers below the member's degree
// (NR of them), so late steps cost a quarter of early ones.
struct Rows4State {
  int hMA, hMB;   // hi(max |coefficient|) of the last two members
  int m12, m13;   // smallest margins of the two step tests so far
  int hmax;       // largest hi(max |t|) so far (finiteness)
  int sp, vp;     // last member positive at +inf (0 / 1); sign changes at +inf
};

// maximum of an int over each 16-lane row, left in every lane of the row
__device__ __forceinline__ int row_max_int(int h) {
  h = max(h, dpp_i<0xB1, 0xf>(h));    // quad_perm [1, 0, 3, 2]
  h = max(h, dpp_i<0x4E, 0xf>(h));    // quad_perm [2, 3, 0, 1]
  h = max(h, dpp_i<0x124, 0xf>(h));   // row_ror:4
  h = max(h, dpp_i<0x128, 0xf>(h));   // row_ror:8
  return h;
}

__device__ __forceinline__ void sturm4_begin(const double (&G)[4], double gtop, int D, int l, double (&A)[4],
                                             double (&B)[4], double& bl, double& ab, Rows4State& S, bool& ok) {
  const double ag = fabs(gtop), sgn = gtop > 0.0 ? 1.0 : -1.0;
  const double sa = fast_rcp_d(ag + 1e-300), sb = fast_rcp_d(D * ag + 1e-300);
  ok = ag > 0.0 && ag < INFINITY;
  int hA = 0, hB = 0;
  double nxt = dpp_d<0x12F>(G[0]);   // row_ror:15: lane l + 1 of the row (lane 0 at l = 15)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = 16 * r + l;
    const double up = r < 3 ? dpp_d<0x12F>(G[r < 3 ? r + 1 : 3]) : 0.0;
    const double g1 = l == 15 ? up : nxt;   // coefficient k + 1
    nxt = up;
    const double dv = k < D ? (k + 1) * g1 : 0.0;
    A[r] = k == D ? sgn : G[r] * sa;
    B[r] = k == D - 1 ? sgn : dv * sb;
    hA = max(hA, hiword(A[r]) & 0x7fffffff);
    hB = max(hB, hiword(B[r]) & 0x7fffffff);
  }
  S.hMA = max(row_max_int(hA), kHi1);
  S.hMB = row_max_int(hB);
  S.m12 = S.m13 = 0x7fffffff;
  S.hmax = 0;
  S.sp = gtop > 0.0 ? 1 : 0;
  S.vp = 0;
  bl = sgn;
  ab = 1.0;
}

// Member q from the last two: A (older, degree db + 1) is overwritten by the
// new member; B (degree db) is the newer.  db = D - q + 1; NR registers hold
// every coefficient up to db + 1, so db itself lies in register NR - 1, or in
// NR - 2 when db + 1 starts register NR - 1 (db % 16 == 15), and db - 1 one
// register lower still when db % 16 == 0.
template <int NR>
__device__ __forceinline__ void sturm4_step(double (&A)[4], const double (&B)[4], double& bl, double& ab,
                                            Rows4State& S, int db, int l, int pbase) {
  double t[NR];
  double below = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double rot = dpp_d<0x121>(B[r]);   // row_ror:1: lane l - 1 (lane 0: lane 15)
    t[r] = fma(-ab, l == 0 ? below : rot, A[r]);
    below = rot;
  }
  const int lq = db & 15;
  const bool top = lq != 15;                          // db in register NR - 1 (else NR - 2)
  const double tq = NR == 1 ? t[0] : (top ? t[NR - 1] : t[NR > 1 ? NR - 2 : 0]);
  const double q0 = bperm_d(pbase + (lq << 2), tq) * bl;
  // remainder: coefficients below db (the rest are zeroed)
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double v = fma(-q0, B[r], t[r]);
    if (r < NR - 2) {
      t[r] = v;
    } else if (r == NR - 2) {
      t[r] = (top || l < lq) ? v : 0.0;
    } else {
      t[r] = (top && l < lq) ? v : 0.0;
    }
  }
  // the new leading coefficient, index db - 1
  const int ll = (db - 1) & 15;
  const int rl = (db - 1) >> 4, rtop = (db + 1) >> 4;   // rtop = NR - 1
  const int drop = rtop - rl;                              // 0, 1 or 2 registers below the top
  double tl = t[NR - 1];
  if (NR > 1) tl = drop == 1 ? t[NR > 1 ? NR - 2 : 0] : tl;
  if (NR > 2) tl = drop == 2 ? t[NR > 2 ? NR - 3 : 0] : tl;
  const double lead = bperm_d(pbase + (ll << 2), tl);
  int h = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) h = max(h, hiword(t[r]) & 0x7fffffff);
  const int hr = row_max_int(h);
  const int hlead = hiword(lead), ha = hlead & 0x7fffffff;
  S.m12 = min(S.m12, hr - max(S.hMA, S.hMB));
  S.m13 = min(S.m13, ha - hr);
  S.hmax = max(S.hmax, hr);
  S.hMA = S.hMB;
  S.hMB = sturm_member_hi(hr, ha);
  const int tp = (int)((unsigned)hlead >> 31);   // P_q = -t / |lead| positive at +inf
  S.vp += tp ^ S.sp;
  S.sp = tp;
  const double sc = fast_rcp_d(fabs(lead) + 1e-300);
  const double nb = from_hiword((hlead & 0x80000000) ^ 0xbff00000);   // -sign(lead)
#pragma unroll
  for (int r = 0; r < NR; ++r) A[r] = -t[r] * sc;
  ab = bl * nb;
  bl = nb;
}

// steps q .. qend - 1 with NR registers; A holds the older member and B the
// newer on entry and on return
template <int NR>
__device__ __forceinline__ void sturm4_phase(double (&A)[4], double (&B)[4], double& bl, double& ab, Rows4State& S,
                                             int D, int& q, int qend, int l, int pbase) {
  for (; q + 1 < qend; q += 2) {
    sturm4_step<NR>(A, B, bl, ab, S, D - q + 1, l, pbase);
    sturm4_step<NR>(B, A, bl, ab, S, D - q, l, pbase);
  }
  if (q < qend) {
    sturm4_step<NR>(A, B, bl, ab, S, D - q + 1, l, pbase);
    ++q;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double x = A[r];
      A[r] = B[r];
      B[r] = x;
    }
  }
}

// Distinct real roots of the degree-D polynomial of this lane's row (D + 1 <=
// 64; G[r] = coefficient 16 r + (lane & 15), zero above D; gtop = coefficient
// D), or -1 when a step fails its test (`raw`: the count regardless).  All
// lanes must be active.
__device__ __forceinline__ int sturm_count_rows4(const double (&G)[4], double gtop, int D, int lane, int& raw) {
  const int l = lane & 15, pbase = (lane & 48) << 2;
  double A[4], B[4], bl, ab;
  Rows4State S;
  bool ok;
  sturm4_begin(G, gtop, D, l, A, B, bl, ab, S, ok);
  // step q touches coefficients up to D - q + 2: four registers while that is
  // at least 48, three down to 32, two down to 16, then one
  int q = 2;
  sturm4_phase<4>(A, B, bl, ab, S, D, q, min(D + 1, D - 45), l, pbase);
  sturm4_phase<3>(A, B, bl, ab, S, D, q, min(D + 1, D - 29), l, pbase);
  sturm4_phase<2>(A, B, bl, ab, S, D, q, min(D + 1, D - 13), l, pbase);
  sturm4_phase<1>(A, B, bl, ab, S, D, q, D + 1, l, pbase);
  ok = ok && S.hmax < 0x7ff00000 && S.m12 > -kHiT12 && S.m13 > -kHiT13;
  raw = D - 2 * S.vp;
  return ok ? raw : -1;
}

// Newton on R(theta) carried out on the Cayley polynomial.  With x = tan((theta
// - phi0) / 2), f(x) = (1 + x^2)^K R(theta), so R'/R = ((1 + x^2) f'/f - 2 K x)
// / 2 and the Newton step of R in theta is d = 2 f / ((1 + x^2) f' - 2 K x f).
// For |x| > 1 the iterate is kept as y = 1 / x and the reversed polynomial
// g(y) = y^D f(1 / y) = (1 + y^2)^K R(theta) serves the same way, with theta
// decreasing in y, so the formula (in g, y) gives -d.  Either way the iterate u
// = x or y has |u| <= 1, and the step (clamped to 0.5 rad as in theta) is
// applied by the tangent addition formula u <- (u - t) / (1 + u t), t = tan(s
// / 2) from its series to fifth order (the clamp bounds the relative error of
// t by 1.3e-5 and it vanishes as the step does, so convergence stays quadratic);
// if the result leaves [-1, 1] its reciprocal is taken and the representation
// flips.  One Newton step costs a real Horner pass of degree D for f and f'
// (2D multiply-adds) in place of K complex multiply-adds for R and R' plus a
// sine and cosine.  cp: coefficients of f (sg > 0) or of g (sg < 0) in
// ascending order.  Returns the signed step s (theta moves by sg * s, clamped);
// ok drops on a zero or non-finite step.
__device__ __forceinline__ double newton_u_step(const double* cp, int D, int K, double& u, int& sg, bool& ok) {
  // f = E(v) + u O(v), v = u^2 (D even: E has the even powers up to D, O the
  // odd ones up to D - 1), f' = 2u E'(v) + O(v) + 2v O'(v): four independent
  // Horner chains of D/2 steps in place of two of D
  const double v = u * u;
  double E = cp[D], dE = 0.0, O = cp[D - 1], dO = 0.0;
  // (the new E and O are formed in the loaded coefficients' registers and the
  // derivatives in the old ones', so no step needs a register copy)
#pragma unroll 4
  for (int c = D - 2; c >= 2; c -= 2) {
    const double a = cp[c], b = cp[c - 1];
    const double nE = fma(E, v, a), nO = fma(O, v, b);
    dE = fma(dE, v, E);
    dO = fma(dO, v, O);
    E = nE;
    O = nO;
  }
  dE = fma(dE, v, E);
  E = fma(E, v, cp[0]);
  const double F = fma(u, O, E);
  const double dF = fma(2.0 * u, dE, fma(2.0 * v, dO, O));
  const double den = fma(fma(u, u, 1.0), dF, -(2.0 * K) * u * F);
  const double d = 2.0 * F * fast_rcp_d(den);
  ok = den != 0.0 && isfinite(d);
  const double sc = fmax(-0.5, fmin(0.5, d));
  const double h = 0.5 * sc, h2 = h * h;
  const double t = h * fma(h2, fma(h2, 0.13333333333333333333, 0.33333333333333333333), 1.0);
  const double num = u - t, dd = fma(u, t, 1.0);
  const bool flip = fabs(num) > fabs(dd);
  u = (flip ? dd : num) * fast_rcp_d(flip ? num : dd);
  sg = flip ? -sg : sg;
  return sc;
}

// Convergence of a Newton lane from its step sizes: a step below 1e-12, or,
// in the quadratic regime, a step small enough that the iterate it produced
// is already within ~1e-14 of the root.  With steps s_{k-1}, s_k and the
// error after step k about C s_k^2, C ~ s_k / s_{k-1}^2, the second test is
// s_k^3 < 1e-14 s_{k-1}^2 (with s_k < 1e-6 and s_{k-1} < 1e-3, so that both
// steps are local ones, not a clamped jump); a slowly (linearly) converging
// lane, as near a double root, passes only the first.  Saves the step that
// would merely confirm convergence.
__device__ __forceinline__ bool newton_settled(double sc, double& prev) {
  const double a = fabs(sc);
  const bool c = a < 1e-12 || (a < 1e-6 && prev < 1e-3 && a * a * a < 1e-14 * prev * prev);
  prev = a;
  return c;
}

// Iterate (u, sg) of the phase whose direction is (c, s) (any length r > 0)
// relative to phi0: tan(alpha / 2) = s / (r + c), taken while c >= 0 (|u| <=
// 1); otherwise its reciprocal, (r + c) / s = s / (r - c).
__device__ __forceinline__ void u_from_dir(double c, double s, double& u, int& sg) {
  const double r = sqrt(fma(c, c, s * s));
  const bool in = c >= 0.0;
  u = s * fast_rcp_d(fmax(in ? r + c : r - c, 1e-300));
  sg = in ? 1 : -1;
}

// atan(u) for |u| <= 1.  Two halvings, atan(u) = 2 atan(u / (1 + sqrt(1 +
// u^2))), bring the argument below tan(pi / 16) < 0.199, where the Taylor
// series through z^23 leaves a remainder below 2e-17 of the result.
// (coefficients (-1)^n / (2n + 1), n = 11 .. 1, read through poly_table)
static __constant__ double kAtanTab[11] = {
    -1.0 / 23.0, 1.0 / 21.0, -1.0 / 19.0, 1.0 / 17.0, -1.0 / 15.0, 1.0 / 13.0,
    -1.0 / 11.0, 1.0 / 9.0,  -1.0 / 7.0,  1.0 / 5.0,  -1.0 / 3.0};
__device__ __forceinline__ double atan_unit(double u) {
  const const_table T = poly_table((const_table)kAtanTab);
  double z = u * fast_rcp_d(1.0 + sqrt(fma(u, u, 1.0)));
  z = z * fast_rcp_d(1.0 + sqrt(fma(z, z, 1.0)));
  const double z2 = z * z;
  double p = T[0];
#pragma unroll
  for (int i = 1; i < 11; ++i) p = fma(p, z2, T[i]);
  return 4.0 * fma(p * z2, z, z);
}

// Phase in [0, 2 pi) of the iterate: phi0 + 2 atan u (sg > 0), phi0 + pi sign(u)
// - 2 atan u (sg < 0).
__device__ __forceinline__ double theta_from_u(double phi0, double u, int sg) {
  const double au = 2.0 * atan_unit(u);
  double th = sg > 0 ? phi0 + au : phi0 + copysign(kPi, u) - au;
  th = fma(-floor(th * (1.0 / kTwoPi)), kTwoPi, th);
  return th >= kTwoPi ? th - kTwoPi : (th < 0.0 ? th + kTwoPi : th);
}

// Four frequencies per wavefront (H <= 10, D < 64): frequencies 4b .. 4b + 3
// of the list.  Their four Sturm chains run side by side, one per 16-lane
// row (sturm_count_rows4); then Newton runs on two of them at a time, lanes
// 0..31 for the first and 32..63 for the second, each half with min(32, D)
// starts: the 2H network seeds and min(32, D) - 2H evenly spaced phases (all
// evenly spaced without network).  The Newton steps are those of R in theta,
// evaluated on the Cayley polynomial (newton_u_step); converged roots are
// merged one root per pass, and a half that has reached its count is frozen
// while the other goes on.
struct NewtonAcc {
  unsigned long long iters, roots, fb;
};

// Newton on frequencies wA (lanes 0..31) and wA + 1 (lanes 32..63, if hasB)
// with Sturm counts cA, cB (-2 inactive, -1 untrusted); f of each half and its
// reversal in fb (LDS, 2 FS doubles per half).
__device__ __forceinline__ void newton_pair(const LearnArgs& L, const RecLayout& RL, int H, int64_t wA, int cA, int cB,
                                            const double* fb, int lane, NewtonAcc& acc) {
  const int half = lane >> 5, hl = lane & 31;
  // starts per frequency: every lane of the half (at most D), or only 2H
  // (flag bit 1: the equal-starts comparison of seeds and evenly spaced phases)
  const int K = 3 * H - 1, D = 2 * K, S = 2 * H, NS = (L.flags & 2u) ? S : (D < 32 ? D : 32);
  const int FS = D + 2;
  const unsigned long long lo32 = 0xffffffffull;
  const unsigned long long hmask = half ? ~lo32 : lo32;
  const unsigned long long below = (1ull << lane) - 1ull;
  if (cA == -2 && cB == -2) return;
  double* Rh = L.rec + (wA + half) * (int64_t)RL.stride;   // this lane's frequency (unused when inactive)
  const int64_t wh = wA + half;
  const int cnt = half ? cB : cA;
  const double phi0 = cnt != -2 ? Rh[RL.meta + M_PHI0] : 0.0;
  double u = 0.0;
  int sg = 1;
  bool conv = false, live = cnt >= 0 && hl < NS;
  int its = 0;
  double prev_step = 1.0;
  if (live) {
    // start direction relative to phi0: a network seed (its output vector
    // is the root's direction in the canonical frame, rotated here by
    // -(canon + phi0)) or an evenly spaced phase less phi0
    const bool seeded = L.seeds_out && hl < S;
    double bc = 1.0, bs = 0.0, ang;
    if (seeded) {
      const float* o = L.seeds_out + wh * 2 * S;
      bc = (double)o[2 * hl];
      bs = (double)o[2 * hl + 1];
      ang = -(Rh[RL.meta + M_CANON] + phi0);
    } else {
      ang = (L.seeds_out ? (hl - S + 0.5) * (kTwoPi / (NS - S)) : (hl + 0.5) * (kTwoPi / NS)) - phi0;
    }
    double s1, c1;
    sincos_small(ang, s1, c1);
    u_from_dir(fma(bc, c1, -bs * s1), fma(bc, s1, bs * c1), u, sg);
  }
  const double* fbase = fb + 2 * FS * half;
  bool doneA = cA < 0, doneB = cB < 0;
  unsigned long long um = 0ull, merged = 0ull, U = 0ull;   // U: unique converged lanes
  for (int it = 1; it <= 12 && !(doneA && doneB); ++it) {
    if (live && !conv) {
      bool ok;
      const double sc = newton_u_step(sg > 0 ? fbase : fbase + FS, D, K, u, sg, ok);
      if (!ok) {
        live = false;
      } else {
        ++its;
        if (newton_settled(sc, prev_step)) conv = true;
      }
    }
    if (it >= 2) {   // merges are incremental, so every iteration from the second checks
      const unsigned long long cm = __ballot(conv);
      const bool needA = !doneA && __popcll(cm & lo32) >= cA;
      const bool needB = !doneB && __popcll(cm >> 32) >= cB;
      if (!needA && !needB && it < 12) continue;
      // distinct converged roots of each half: a converged lane is unique
      // unless a lower converged lane of its half lies within 1e-8 rad.
      // Compared on key = u (sg > 0) or sign(u) 2 - u (sg < 0), which
      // increases with theta - phi0 over (-pi, pi) and moves by |du| where
      // theta moves by 2 |du| / (1 + u^2) (the cut at theta - phi0 = pi
      // sits where R is largest, far from any root).  Converged lanes no
      // longer move, so each check settles only the lanes converged since
      // the last: one pass per root, from the lowest pending lane jj, marks
      // every converged lane of its half within the tolerance of jj; jj is
      // unique if none of them is lower, and the higher ones (also roots
      // settled earlier) are not.
      const double key = sg > 0 ? u : copysign(2.0, u) - u;
      for (unsigned long long pend = cm & ~merged; pend;) {
        const int jj = __builtin_ctzll(pend);
        const double kj = lrdlane(key, jj), uj = lrdlane(u, jj);
        const double tol = 0.5e-8 * fma(uj, uj, 1.0);
        const unsigned long long bit = 1ull << jj;
        const unsigned long long same = __ballot(fabs(key - kj) < tol) & cm & (jj < 32 ? lo32 : ~lo32);
        const unsigned long long upto = (bit << 1) - 1ull;   // lanes 0..jj
        U &= upto | ~same;
        U = (same & (bit - 1ull)) ? (U & ~bit) : (U | bit);
        pend &= ~(same | bit);
      }
      merged = cm;
      um = U;
      if (__popcll(um & lo32) == cA) doneA = true;
      if (__popcll(um >> 32) == cB) doneB = true;
      if (half ? doneB : doneA) live = false;
    }
  }
  acc.iters += (unsigned long long)wave_sum((double)its);
  const double thw = theta_from_u(phi0, u, sg);
  const int nuA = __popcll(um & lo32), nuB = __popcll(um >> 32);
  const bool okA = cA >= 0 && nuA == cA, okB = cB >= 0 && nuB == cB;
  const bool ok = half ? okB : okA;
  const int nu = half ? nuB : nuA;
  double* cand = Rh + RL.cand;
  if (cnt != -2 && ok)
    for (int c = hl; c < D; c += 32) cand[c] = __longlong_as_double(0x7ff8000000000000ll);
  lwave_sync();
  // confirmed roots, or the distinct roots found, which start the Aberth
  // iteration of a fallback frequency
  if (cnt != -2 && ((um >> lane) & 1ull)) cand[__popcll(um & hmask & below)] = thw;
  if (cnt != -2 && !ok && hl == 0) {
    Rh[RL.meta + M_WARM] = (double)nu;
    Rh[RL.meta + M_COUNT] = (double)cnt;
    Rh[RL.meta + M_FALLBACK] = 1.0;
    const unsigned slot = atomicAdd(L.fb_count, 1u);
    L.fb_list[slot] = wh;
  }
  acc.roots += (unsigned long long)((okA ? nuA : 0) + (okB ? nuB : 0));
  acc.fb += (unsigned long long)((cA != -2 && !okA) + (cB != -2 && !okB));
  lwave_sync();
}

// OCC: resident wavefronts per SIMD the register allocation is made for (4:
// up to 128 VGPRs; 5: up to 96, a few spills outside the Newton loop; 6: up
// to 80, more spills, but more waves to cover the Sturm steps' latency);
// which is faster depends on the workload and the grid, so the launch shape
// picks it.
template <int OCC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC))) void k_newton_sturm4(SolveArgs a, LearnArgs L) {
  extern __shared__ double sml[];
  const int lane = threadIdx.x & 63, row = lane >> 4, l = lane & 15;
  const int H = a.H, D = 6 * H - 2;
  const int FS = D + 2;   // f and its reversal for each frequency, 16-byte aligned
  const RecLayout RL(H);
  NewtonAcc acc{0, 0, 0};
  for (int64_t w0 = 4 * (int64_t)blockIdx.x; w0 < L.np; w0 += 4 * (int64_t)gridDim.x) {
    // statuses of the four frequencies (inactive: past the end, rejected
    // lightcurve, or P constant in theta_2)
    int act = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (w0 + c < L.np) {
        const int st = (int)L.rec[(w0 + c) * (int64_t)RL.stride + RL.meta + M_STATUS];
        act |= (st != ST_BAD_LC && st != ST_CONSTANT) ? 1 << c : 0;
      }
    }
    if (!act) continue;
    if (L.flags & 1u) {   // forced fallback
      if (l == 0 && ((act >> row) & 1)) {
        const unsigned slot = atomicAdd(L.fb_count, 1u);
        L.fb_list[slot] = w0 + row;
        double* Rr = L.rec + (w0 + row) * (int64_t)RL.stride;
        Rr[RL.meta + M_FALLBACK] = 1.0;
        Rr[RL.meta + M_WARM] = 0.0;
        Rr[RL.meta + M_COUNT] = -1.0;
      }
      acc.fb += (unsigned long long)__popc((unsigned)act);
      continue;
    }
    // lane 16 c + l: coefficients 16 r + l of frequency c (zero above D or
    // for an inactive frequency); f and its reversal to LDS for Newton
    const bool mine = (act >> row) & 1;
    const double* f = L.rec + (w0 + (mine ? row : 0)) * (int64_t)RL.stride + RL.f;
    double G[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 16 * r + l;
      G[r] = (mine && k <= D) ? f[k] : 0.0;
      if (mine && k <= D) {
        sml[2 * FS * row + k] = G[r];
        sml[2 * FS * row + FS + D - k] = G[r];
      }
    }
    const double gtop = mine ? f[D] : 0.0;
    lwave_sync();
    int raw;
    int cnt = sturm_count_rows4(G, gtop, D, lane, raw);
    if (cnt < 2) cnt = -1;
    if (!mine) cnt = -2;
    const int c0 = __builtin_amdgcn_readlane(cnt, 0), c1 = __builtin_amdgcn_readlane(cnt, 16);
    const int c2 = __builtin_amdgcn_readlane(cnt, 32), c3 = __builtin_amdgcn_readlane(cnt, 48);
#pragma unroll 1
    for (int p = 0; p < 2; ++p) newton_pair(L, RL, H, w0 + 2 * p, p ? c2 : c0, p ? c3 : c1, sml + 4 * FS * p, lane, acc);
  }
  if (lane == 0 && a.counters) {
    SolveCounters* c = counter_slot(a.counters);
    if (acc.iters) atomicAdd(&c->newton_iters, acc.iters);
    if (acc.roots) atomicAdd(&c->roots_found, acc.roots);
    if (acc.fb) atomicAdd(&c->fallback, acc.fb);
  }
}

// One frequency per wavefront (H = 11, D = 64): the Sturm chain of f in
// registers (the degree-64 coefficient as a scalar), then Newton from 4H
// starts (the 2H network seeds and 2H evenly spaced phases; all evenly spaced
// without network), stepped on the Cayley polynomial and merged one root per
// pass as in k_newton_sturm4, with the same stop rule.
__host__ __device__ inline size_t learn_lds_bytes(int H) {
  const int D = 6 * H - 2;
  return (size_t)(2 * (D + 2)) * sizeof(double);   // f and its reversal
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_newton_sturm(SolveArgs a, LearnArgs L) {
  extern __shared__ double sml[];
  const int lane = threadIdx.x & 63;
  const int H = a.H, K = 3 * H - 1, D = 2 * K, S = 2 * H, NS = 2 * S;
  const int FS = D + 2;
  const RecLayout RL(H);
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned long long iters_acc = 0, roots_acc = 0, fb_acc = 0;
  for (int64_t w = first_item(L.queue, lane); w < L.np; w = next_item(L.queue, lane, w)) {
    double* R = L.rec + w * (int64_t)RL.stride;
    const int st = (int)R[RL.meta + M_STATUS];
    if (st == ST_BAD_LC || st == ST_CONSTANT) continue;
    if (L.flags & 1u) {   // forced fallback
      if (lane == 0) {
        const unsigned slot = atomicAdd(L.fb_count, 1u);
        L.fb_list[slot] = w;
        R[RL.meta + M_FALLBACK] = 1.0;
        R[RL.meta + M_WARM] = 0.0;
        R[RL.meta + M_COUNT] = -1.0;
      }
      ++fb_acc;
      continue;
    }
    for (int c = lane; c <= D; c += 64) {
      const double fc = R[RL.f + c];
      sml[c] = fc;
      sml[FS + D - c] = fc;
    }
    const double gv = lane <= D ? R[RL.f + lane] : 0.0;
    const double gv1 = lane + 64 <= D ? R[RL.f + 64 + lane] : 0.0;
    const double gtop = R[RL.f + D];
    lwave_sync();
    // Sturm count first: an ill-determined count (or fewer than the two real
    // roots every non-constant P has) sends the frequency on without Newton
    int raw;
    int cnt = D > 64 ? sturm_count_dd(gv, gv1, D, lane, raw) : sturm_count_line_reg(gv, gtop, D, lane, raw);
    if (cnt < 2) cnt = -1;
    const double phi0 = R[RL.meta + M_PHI0];
    double u = 0.0;
    int sg = 1;
    bool conv = false, live = cnt >= 0 && lane < NS;
    int its = 0;
    double prev_step = 1.0;
    if (live) {
      const bool seeded = L.seeds_out && lane < S;
      double bc = 1.0, bs = 0.0, ang;
      if (seeded) {
        const float* o = L.seeds_out + w * 2 * S;
        bc = (double)o[2 * lane];
        bs = (double)o[2 * lane + 1];
        ang = -(R[RL.meta + M_CANON] + phi0);
      } else {
        ang = (L.seeds_out ? (lane - S + 0.5) * (kTwoPi / (NS - S)) : (lane + 0.5) * (kTwoPi / NS)) - phi0;
      }
      double s1, c1;
      sincos_small(ang, s1, c1);
      u_from_dir(fma(bc, c1, -bs * s1), fma(bc, s1, bs * c1), u, sg);
    }
    bool done = cnt < 0;
    unsigned long long um = 0ull, merged = 0ull, U = 0ull;
    for (int it = 1; it <= 12 && !done; ++it) {
      if (live && !conv) {
        bool ok;
        const double sc = newton_u_step(sg > 0 ? sml : sml + FS, D, K, u, sg, ok);
        if (!ok) {
          live = false;
        } else {
          ++its;
          if (newton_settled(sc, prev_step)) conv = true;
        }
      }
      if (it >= 2) {
        const unsigned long long cm = __ballot(conv);
        // fewer converged lanes than the count cannot reach it (the last
        // check always runs: its roots seed the fallback)
        if (__popcll(cm) < cnt && it < 12) continue;
        const double key = sg > 0 ? u : copysign(2.0, u) - u;
        for (unsigned long long pend = cm & ~merged; pend;) {
          const int jj = __builtin_ctzll(pend);
          const double kj = lrdlane(key, jj), uj = lrdlane(u, jj);
          const double tol = 0.5e-8 * fma(uj, uj, 1.0);
          const unsigned long long bit = 1ull << jj;
          const unsigned long long same = __ballot(fabs(key - kj) < tol) & cm;
          const unsigned long long upto = (bit << 1) - 1ull;
          U &= upto | ~same;
          U = (same & (bit - 1ull)) ? (U & ~bit) : (U | bit);
          pend &= ~(same | bit);
        }
        merged = cm;
        um = U;
        if (__popcll(um) == cnt) {
          done = true;
          live = false;
        }
      }
    }
    iters_acc += (unsigned long long)wave_sum((double)(lane < NS ? its : 0));
    const double thw = theta_from_u(phi0, u, sg);
    const int nu = __popcll(um);
    const bool uniq = (um >> lane) & 1ull;
    if (cnt >= 0 && cnt == nu) {
      double* cand = R + RL.cand;
      for (int c = lane; c < D; c += 64) cand[c] = __longlong_as_double(0x7ff8000000000000ll);
      lwave_sync();
      if (uniq) cand[__popcll(um & below)] = thw;
      roots_acc += (unsigned long long)nu;
    } else {
      // the distinct roots Newton did find start the Aberth iteration
      if (uniq) R[RL.cand + __popcll(um & below)] = thw;
      if (lane == 0) {
        R[RL.meta + M_WARM] = (double)nu;
        R[RL.meta + M_COUNT] = (double)cnt;
        R[RL.meta + M_FALLBACK] = 1.0;
        const unsigned slot = atomicAdd(L.fb_count, 1u);
        L.fb_list[slot] = w;
      }
      ++fb_acc;
    }
    lwave_sync();
  }
  if (lane == 0 && a.counters) {
    SolveCounters* c = counter_slot(a.counters);
    if (iters_acc) atomicAdd(&c->newton_iters, iters_acc);
    if (roots_acc) atomicAdd(&c->roots_found, roots_acc);
    if (fb_acc) atomicAdd(&c->fallback, fb_acc);
  }
}

// Root counts of a record chunk (diagnostic of the count the learned and
// uniform solvers trust): per pair, the Sturm count of the Cayley polynomial
// f by the device code the Newton kernels use (sturm_count_rows4, four pairs
// per wavefront, for H <= 10; sturm_count_line_reg for H = 11,
// sturm_count_dd above), -1000 - n when the
// chain fails its test (n: the count it reached regardless), -2 for an
// inactive pair; and the number of real
// eigenvalues the companion QR (run before this kernel) marked in M_REAL_LO,
// M_REAL_HI and M_REAL_X (-1 when the QR did not converge).
__global__ __launch_bounds__(64) void k_root_counts(const double* rec, int H, int64_t np, int* sturm, int* real) {
  const int lane = threadIdx.x & 63;
  const int D = 6 * H - 2;
  const RecLayout RL(H);
  const bool four = D < 64;
  const int64_t per = four ? 4 : 1;
  for (int64_t w0 = per * (int64_t)blockIdx.x; w0 < np; w0 += per * (int64_t)gridDim.x) {
    int cnt;
    if (four) {
      const int row = lane >> 4, l = lane & 15;
      const bool in = w0 + row < np;
      const double* f = rec + (w0 + (in ? row : 0)) * (int64_t)RL.stride + RL.f;
      double G[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) G[r] = (in && 16 * r + l <= D) ? f[16 * r + l] : 0.0;
      int raw;
      cnt = sturm_count_rows4(G, in ? f[D] : 0.0, D, lane, raw);
      if (cnt < 0) cnt = -1000 - raw;
      cnt = __builtin_amdgcn_readlane(cnt, 0) * (lane == 0) + __builtin_amdgcn_readlane(cnt, 16) * (lane == 1) +
            __builtin_amdgcn_readlane(cnt, 32) * (lane == 2) + __builtin_amdgcn_readlane(cnt, 48) * (lane == 3);
    } else {
      const double* RA = rec + w0 * (int64_t)RL.stride;
      const double gv = RA[RL.f + lane];
      const double gv1 = lane + 64 <= D ? RA[RL.f + 64 + lane] : 0.0;
      int raw;
      cnt = D > 64 ? sturm_count_dd(gv, gv1, D, lane, raw) : sturm_count_line_reg(gv, RA[RL.f + D], D, lane, raw);
      if (cnt < 0) cnt = -1000 - raw;
    }
    if (lane < per && w0 + lane < np) {
      const double* Rq = rec + (w0 + lane) * (int64_t)RL.stride;
      const int st = (int)Rq[RL.meta + M_STATUS];
      const bool act = st != ST_BAD_LC && st != ST_CONSTANT;
      const unsigned lo = (unsigned)Rq[RL.meta + M_REAL_LO], hi = (unsigned)Rq[RL.meta + M_REAL_HI];
      const unsigned x = D > 64 ? (unsigned)Rq[RL.meta + M_REAL_X] : 0u;
      const int nreal = __popcll(((unsigned long long)hi << 32) | lo) + __popc(x);
      sturm[w0 + lane] = act ? cnt : -2;
      real[w0 + lane] = act ? (st == ST_NO_CONVERGE ? -1 : nreal) : -2;
    }
  }
}

hipError_t launch_root_counts(const double* rec, int H, int64_t np, int* sturm, int* real, int waves,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_root_counts, dim3((unsigned)waves), dim3(64), 0, st, rec, H, np, sturm, real);
  return hipGetLastError();
}

// Second Newton round (project addition) for the frequencies the first left
// unconfirmed: one frequency per wavefront.  Lanes 0..nu - 1 hold the nu
// distinct roots the first round found (converged, not stepped); lanes
// nu..63 start from new phases: the network's 2H seeds first when the
// learned solver supplies them (row i of `seeds` for list entry i), then
// evenly spaced phases offset from the first round's grid.  Newton steps, the
// merge of converged roots and the stop rule are those of the first round,
// against the Sturm count it kept in M_COUNT; a frequency that reaches its
// count is settled (its roots become the candidates), the others go on to
// the Aberth tier through out_list with the roots found as its warm start.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_newton_retry(RetryArgs A) {
  // the fallback tiers run beside the side stream's scoring: their waves
  // take issue priority over it on a shared SIMD (the tiers are few, latency-bound
  // waves on the step's critical path)
  __builtin_amdgcn_s_setprio(2);
  extern __shared__ double sml[];
  const int lane = threadIdx.x & 63;
  const int H = A.H, K = 3 * H - 1, D = 2 * K, S = 2 * H;
  const int FS = D + 2;
  const RecLayout RL(H);
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t n = (int64_t)*A.count;
  unsigned long long iters_acc = 0, left_acc = 0;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t w = A.list[i];
    double* R = A.rec + w * (int64_t)RL.stride;
    const int cnt = (int)R[RL.meta + M_COUNT];
    if (cnt < 2) {   // no trusted count (or a forced fallback): straight on
      if (lane == 0) {
        const unsigned slot = atomicAdd(A.out_count, 1u);
        A.out_list[slot] = w;
      }
      ++left_acc;
      continue;
    }
    for (int c = lane; c <= D; c += 64) {
      const double fc = R[RL.f + c];
      sml[c] = fc;
      sml[FS + D - c] = fc;
    }
    const int nu0 = (int)R[RL.meta + M_WARM];
    const double phi0 = R[RL.meta + M_PHI0];
    lwave_sync();
    double u = 0.0;
    int sg = 1;
    bool conv = false, live = false;
    int its = 0;
    double prev_step = 1.0;
    {
      double bc = 1.0, bs = 0.0, ang;
      const int k = lane - nu0, nst = 64 - nu0;
      if (lane < nu0) {
        ang = R[RL.cand + lane] - phi0;   // a root the first round found
        conv = true;
      } else if (A.seeds && k < S) {
        const float* o = A.seeds + i * 2 * S;
        bc = (double)o[2 * k];
        bs = (double)o[2 * k + 1];
        ang = -(R[RL.meta + M_CANON] + phi0);
        live = true;
      } else {
        const int kk = A.seeds ? k - S : k, nn = A.seeds ? nst - S : nst;
        ang = (kk + 0.25) * (kTwoPi / nn) - phi0;
        live = true;
      }
      double s1, c1;
      sincos_small(ang, s1, c1);
      u_from_dir(fma(bc, c1, -bs * s1), fma(bc, s1, bs * c1), u, sg);
    }
    bool done = false;
    unsigned long long um = 0ull, merged = 0ull, U = 0ull;
    for (int it = 1; it <= 12 && !done; ++it) {
      if (live && !conv) {
        bool ok;
        const double sc = newton_u_step(sg > 0 ? sml : sml + FS, D, K, u, sg, ok);
        if (!ok) {
          live = false;
        } else {
          ++its;
          if (newton_settled(sc, prev_step)) conv = true;
        }
      }
      const unsigned long long cm = __ballot(conv);
      if (__popcll(cm) < cnt && it < 12) continue;
      const double key = sg > 0 ? u : copysign(2.0, u) - u;
      for (unsigned long long pend = cm & ~merged; pend;) {
        const int jj = __builtin_ctzll(pend);
        const double kj = lrdlane(key, jj), uj = lrdlane(u, jj);
        const double tol = 0.5e-8 * fma(uj, uj, 1.0);
        const unsigned long long bit = 1ull << jj;
        const unsigned long long same = __ballot(fabs(key - kj) < tol) & cm;
        const unsigned long long upto = (bit << 1) - 1ull;
        U &= upto | ~same;
        U = (same & (bit - 1ull)) ? (U & ~bit) : (U | bit);
        pend &= ~(same | bit);
      }
      merged = cm;
      um = U;
      if (__popcll(um) == cnt) done = true;
    }
    iters_acc += (unsigned long long)wave_sum((double)its);
    const double thw = theta_from_u(phi0, u, sg);
    const int nu = __popcll(um);
    const bool uniq = (um >> lane) & 1ull;
    lwave_sync();
    if (done) {
      double* cand = R + RL.cand;
      for (int c = lane; c < D; c += 64) cand[c] = __longlong_as_double(0x7ff8000000000000ll);
      lwave_sync();
      if (uniq) cand[__popcll(um & below)] = thw;
    } else {
      if (uniq) R[RL.cand + __popcll(um & below)] = thw;
      if (lane == 0) {
        R[RL.meta + M_WARM] = (double)nu;
        const unsigned slot = atomicAdd(A.out_count, 1u);
        A.out_list[slot] = w;
      }
      ++left_acc;
    }
    lwave_sync();
  }
  if (lane == 0 && A.counters) {
    SolveCounters* c = counter_slot(A.counters);
    if (iters_acc) atomicAdd(&c->newton_iters, iters_acc);
    if (left_acc) atomicAdd(&c->fallback_aberth, left_acc);
  }
}

hipError_t launch_newton_retry(const RetryArgs& A, int waves, hipStream_t st) {
  hipLaunchKernelGGL(k_newton_retry, dim3((unsigned)waves), dim3(64), learn_lds_bytes(A.H), st, A);
  return hipGetLastError();
}

bool newton_four_per_wave(int H) { return 6 * H - 2 < 64; }

// `done` (nullable): an event the launch itself records at the kernel's end
// (no marker packet of its own on the stream); `occ`: 4, 5 or 6 (k_newton_sturm4).
hipError_t launch_newton_sturm(const SolveArgs& a, const LearnArgs& L, int waves, int occ, hipStream_t st,
                               hipEvent_t done) {
  if (newton_four_per_wave(a.H)) {
    const size_t lds = (size_t)8 * (6 * a.H) * sizeof(double);   // 8 x (D + 2): f and its reversal, four pairs
    if (occ == 6)
      hipExtLaunchKernelGGL(k_newton_sturm4<6>, dim3((unsigned)waves), dim3(64), lds, st, nullptr, done, 0, a, L);
    else if (occ == 5)
      hipExtLaunchKernelGGL(k_newton_sturm4<5>, dim3((unsigned)waves), dim3(64), lds, st, nullptr, done, 0, a, L);
    else
      hipExtLaunchKernelGGL(k_newton_sturm4<4>, dim3((unsigned)waves), dim3(64), lds, st, nullptr, done, 0, a, L);
  } else {
    hipExtLaunchKernelGGL(k_newton_sturm, dim3((unsigned)waves), dim3(64), learn_lds_bytes(a.H), st, nullptr, done, 0,
                          a, L);
  }
  return hipGetLastError();
}

}  // namespace ftp
