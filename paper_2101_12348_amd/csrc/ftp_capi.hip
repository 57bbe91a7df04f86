// Host runtime and C ABI of the fast template periodogram library.
//
// A call runs, on the caller's stream and without host round trips:
//   k_prep_stats -> k_prep_points (+tile histogram) -> scan -> k_bin_fill ->
//   k_spread -> k_fft_pass (1-3 rounds) -> per-frequency solve.
// Lightcurves are processed in chunks whose NFFT grids fit the plan's grid
// budget; a single lightcurve is a chunk of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ftp.h"
#include "ftp_internal.h"
#include "ftp_solve_common.h"
#include "ftp_args.h"

namespace ftp {
// kernels (defined in the other translation units)
__global__ void k_prep_stats(LcInfo*, const double*, const double*, const double*, double*, unsigned*, unsigned*,
                             unsigned*, int64_t);
__global__ void k_sp_combine(LcInfo*, int, const double2*, int);
template <typename R>
__global__ void k_prep_points(const LcInfo*, int64_t, const int64_t*, int64_t, const double*, const double*,
                              const double*, PointRec<R>*, PointRec<R>*, unsigned int*);
__global__ void k_scan_blocks(const unsigned int*, int64_t, int64_t*, int64_t*);
__global__ void k_scan_single(const unsigned int*, int64_t, int64_t*, int64_t*);
__global__ void k_scan_sums(int64_t*, int64_t);
__global__ void k_scan_add(int64_t*, int64_t, const int64_t*, const unsigned int*, int64_t*);
template <typename R>
__global__ void k_bin_fill(const LcInfo*, int64_t, const int64_t*, int64_t, const PointRec<R>*,
                           const PointRec<R>*, const int64_t*, unsigned int*, int*);
template <typename R>
__global__ void k_spread(const LcInfo*, int64_t, const int64_t*, const PointRec<R>*, const PointRec<R>*,
                         const int64_t*, const int*, typename Cplx<R>::T*);
template <typename R>
__global__ void k_fft_pass(const FftGridPass*, int64_t, const int64_t*, const typename Cplx<R>::T*,
                           typename Cplx<R>::T*, const int64_t*);
hipError_t launch_qr(int H, double* rec, int stride, int64_t np, const int64_t* list, const unsigned* list_count,
                     SolveCounters* counters, unsigned* queue, int waves, hipStream_t st);
hipError_t launch_assemble(int precision, const SolveArgs& a, double* rec, int64_t p0, int64_t np, int waves,
                           hipStream_t st);
hipError_t launch_score(const SolveArgs& a, const double* rec, int64_t p0, int64_t np, int waves,
                        hipStream_t st, const int64_t* list = nullptr, const unsigned* list_n = nullptr);
hipError_t launch_score_newton(const SolveArgs& a, const double* rec, int64_t p0, int64_t np, int waves, hipStream_t st,
                         hipEvent_t done = nullptr);
hipError_t launch_gather_sums(int precision, const SolveArgs& a, double* out, int blocks, hipStream_t st);
hipError_t launch_export_stats(const LcInfo* lcs, double* out, hipStream_t st);
struct GemmArgs {
  const uint16_t* A; int64_t a_m, a_k;
  const uint16_t* B; int64_t b_k, b_n;
  int64_t M; int N, K;
  const float* bias;
  const uint16_t* mask; int64_t ld_mask;
  int relu;
  float* Cf; int64_t ld_cf;
  uint16_t* Cb; int64_t ld_cb;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);
hipError_t launch_dense(const uint16_t* A, int64_t lda, const uint16_t* W, int ldw, const float* bias, int64_t M,
                        int N, int Kp, int relu, uint16_t* Yb, float* Yf, int64_t ldy, hipStream_t st);
hipError_t launch_colsum(const float* G, int64_t M, int N, int64_t ld, float* out, hipStream_t st);
hipError_t launch_chamfer(const float* out, int64_t B, int Kseeds, const float* roots, const int* nroots, int R,
                          float lam, float* loss_b, float* dout, uint16_t* dout_bf, hipStream_t st);
hipError_t launch_adam(float* w, uint16_t* wb, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t launch_f32_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t st);
hipError_t launch_features(double* rec, int H, int64_t np, uint16_t* X, int64_t ldx, int waves, hipStream_t st,
                           const int64_t* list = nullptr, const unsigned* list_count = nullptr);
hipError_t launch_newton_retry(const RetryArgs& A, int waves, hipStream_t st);
hipError_t launch_labels(const double* rec, int H, int64_t np, float* roots, int* nroots, int Rmax, int waves,
                         hipStream_t st);
hipError_t launch_root_counts(const double* rec, int H, int64_t np, int* sturm, int* real, int waves,
                              hipStream_t st);
bool newton_four_per_wave(int H);
hipError_t launch_newton_sturm(const SolveArgs& a, const LearnArgs& L, int waves, int occ, hipStream_t st,
                               hipEvent_t done = nullptr);
hipError_t launch_aberth(const AberthArgs& A, int waves, hipStream_t st);
bool mlp_fused_ok(const int* nin, const int* nout);
hipError_t launch_mlp_fused(const FusedMlpArgs& fa, hipStream_t st, int max_blocks = 0, hipEvent_t done = nullptr);
hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t st, unsigned* p2 = nullptr);
hipError_t launch_lc_chi2(const LcInfo* lcs, int64_t n_lc, double* out, hipStream_t st);
hipError_t launch_mb_combine(const double* bp, int64_t n_band, int64_t n_f, const double* chi2, double* power,
                             hipStream_t st);
}  // namespace ftp

using namespace ftp;
static_assert(kFlagPositiveAmp == FTP_FLAG_POSITIVE_AMP, "flag values must agree");

static thread_local std::string g_last_error;

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) {                                                  \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(_e);      \
      return FTP_E_HIP;                                                      \
    }                                                                        \
  } while (0)

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes) {
    if (bytes <= cap) return FTP_OK;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      cap = 0;
      if (e != hipSuccess) { g_last_error = hipGetErrorString(e); return FTP_E_HIP; }
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) { g_last_error = std::string("hipMalloc: ") + hipGetErrorString(e); return FTP_E_HIP; }
    cap = want;
    return FTP_OK;
  }
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
  void release() { if (p) (void)hipFree(p); p = nullptr; cap = 0; }
};

int ilog2_ceil(int64_t v) {
  int l = 0;
  while ((1LL << l) < v) ++l;
  return l;
}

}  // namespace


// Root-proposal network: parameters W1, b1, ..., W4, b4 (W stored (out, in)
// row-major) as FP32 masters with bf16 copies, Adam moments, and the
// activation buffers of the last batch.
struct MlpNet {
  int din = 0, width = 0, dout = 0;
  int64_t n_params = 0;
  int64_t oW[4], ob[4];
  int nin[4], nout[4];
  DevBuf w32, wbf, grad, am, av, loss;
  // inference copy of the bf16 weights with each layer's rows zero-padded to
  // kp[l] (a multiple of 32) and their number to a multiple of 16, for the
  // dense-layer and fused network kernels; built when a plan
  // loads a network whose width is a multiple of 32
  DevBuf winf;
  int kp[4] = {0, 0, 0, 0};
  int64_t oWi[4] = {0, 0, 0, 0};
  bool dense = false;
  DevBuf xbf, h[3], outf, dout_f, dout_b, dz_f, dz_b[2];
  int64_t cap_batch = 0;
  int64_t step = 0;

  void layout() {
    nin[0] = din; nout[0] = width;
    nin[1] = width; nout[1] = width;
    nin[2] = width; nout[2] = width;
    nin[3] = width; nout[3] = dout;
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) {
      oW[l] = o; o += (int64_t)nin[l] * nout[l];
      ob[l] = o; o += nout[l];
    }
    n_params = o;
  }
  int ensure_batch(int64_t B) {
    if (B <= cap_batch) return FTP_OK;
    int rc;
    if ((rc = xbf.ensure(sizeof(uint16_t) * B * din))) return rc;
    for (int l = 0; l < 3; ++l)
      if ((rc = h[l].ensure(sizeof(uint16_t) * B * width))) return rc;
    if ((rc = outf.ensure(sizeof(float) * B * dout))) return rc;
    if ((rc = dout_f.ensure(sizeof(float) * B * dout))) return rc;
    if ((rc = dout_b.ensure(sizeof(uint16_t) * B * dout))) return rc;
    if ((rc = dz_f.ensure(sizeof(float) * B * width))) return rc;
    for (int l = 0; l < 2; ++l)
      if ((rc = dz_b[l].ensure(sizeof(uint16_t) * B * width))) return rc;
    if ((rc = loss.ensure(sizeof(float) * B))) return rc;
    cap_batch = B;
    return FTP_OK;
  }
  void release() {
    DevBuf* bs[] = {&winf, &w32, &wbf, &grad, &am, &av, &loss, &xbf, &h[0], &h[1], &h[2], &outf, &dout_f, &dout_b,
                    &dz_f, &dz_b[0], &dz_b[1]};
    for (DevBuf* b : bs) b->release();
  }
};

uint16_t host_f2bf(float x) {
  unsigned u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Copies FP32 parameters (host) into the net and refreshes the bf16 copies.
int mlp_set_weights(MlpNet* N, const float* w) {
  int rc;
  if ((rc = N->w32.ensure(sizeof(float) * N->n_params))) return rc;
  if ((rc = N->wbf.ensure(sizeof(uint16_t) * N->n_params))) return rc;
  std::vector<uint16_t> b(N->n_params);
  for (int64_t i = 0; i < N->n_params; ++i) b[i] = host_f2bf(w[i]);
  HIP_TRY(hipMemcpy(N->w32.p, w, sizeof(float) * N->n_params, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(N->wbf.p, b.data(), sizeof(uint16_t) * N->n_params, hipMemcpyHostToDevice));
  return FTP_OK;
}

// Padded inference weights (see MlpNet::winf) from host FP32 parameters.
int mlp_build_inference(MlpNet* N, const float* w) {
  N->dense = N->width % 32 == 0;
  if (!N->dense) return FTP_OK;
  // rows padded with zeros to a multiple of 16 (whole MFMA column tiles: the
  // fused network kernel reads every row of a tile unconditionally)
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    N->kp[l] = (N->nin[l] + 31) & ~31;
    N->oWi[l] = o;
    o += (int64_t)((N->nout[l] + 15) & ~15) * N->kp[l];
  }
  std::vector<uint16_t> b((size_t)o, 0);
  for (int l = 0; l < 4; ++l)
    for (int n = 0; n < N->nout[l]; ++n)
      for (int k = 0; k < N->nin[l]; ++k)
        b[N->oWi[l] + (int64_t)n * N->kp[l] + k] = host_f2bf(w[N->oW[l] + (int64_t)n * N->nin[l] + k]);
  int rc;
  if ((rc = N->winf.ensure(sizeof(uint16_t) * (size_t)o))) return rc;
  HIP_TRY(hipMemcpy(N->winf.p, b.data(), sizeof(uint16_t) * (size_t)o, hipMemcpyHostToDevice));
  return FTP_OK;
}

// Inference forward pass with the dense-layer kernel: X (B x kp[0] bf16, row
// stride ldx, zero-padded), hidden activations into N->h[0..2], FP32 output
// (row stride dout).  Same rounding points and K order as mlp_forward.
int mlp_forward_dense(MlpNet* N, const uint16_t* X, int64_t ldx, int64_t B, float* out, hipStream_t st) {
  const uint16_t* wi = N->winf.as<uint16_t>();
  const float* w32 = N->w32.as<float>();
  const uint16_t* in = X;
  int64_t ldin = ldx;
  for (int l = 0; l < 4; ++l) {
    const bool last = l == 3;
    HIP_TRY(launch_dense(in, ldin, wi + N->oWi[l], N->kp[l], w32 + N->ob[l], B, N->nout[l], N->kp[l], last ? 0 : 1,
                         last ? nullptr : N->h[l].as<uint16_t>(), last ? out : nullptr,
                         last ? (int64_t)N->dout : (int64_t)N->width, st));
    if (!last) { in = N->h[l].as<uint16_t>(); ldin = N->width; }
  }
  return FTP_OK;
}

// Forward pass on bf16 inputs X (B x din, row stride din): hidden activations
// into N->h[0..2] (bf16), output (FP32) into out (row stride dout).
int mlp_forward(MlpNet* N, const uint16_t* X, int64_t B, float* out, hipStream_t st) {
  const uint16_t* wb = N->wbf.as<uint16_t>();
  const float* w32 = N->w32.as<float>();
  const uint16_t* in = X;
  int64_t ldin = N->din;
  for (int l = 0; l < 4; ++l) {
    GemmArgs g{};
    g.A = in; g.a_m = ldin; g.a_k = 1;
    g.B = wb + N->oW[l]; g.b_k = 1; g.b_n = N->nin[l];
    g.M = B; g.N = N->nout[l]; g.K = N->nin[l];
    g.bias = w32 + N->ob[l];
    if (l < 3) {
      g.relu = 1;
      g.Cb = N->h[l].as<uint16_t>(); g.ld_cb = N->width;
    } else {
      g.Cf = out; g.ld_cf = N->dout;
    }
    HIP_TRY(launch_gemm(g, st));
    if (l < 3) { in = N->h[l].as<uint16_t>(); ldin = N->width; }
  }
  return FTP_OK;
}

// Loss and gradients (into N->grad) for a batch; forward pass included.
int mlp_loss_grad(MlpNet* N, const uint16_t* X, int64_t B, const float* roots, const int* nroots, int R, float lam,
                  hipStream_t st) {
  int rc;
  if ((rc = N->ensure_batch(B))) return rc;
  if ((rc = N->grad.ensure(sizeof(float) * N->n_params))) return rc;
  if ((rc = mlp_forward(N, X, B, N->outf.as<float>(), st))) return rc;
  HIP_TRY(launch_chamfer(N->outf.as<float>(), B, N->dout / 2, roots, nroots, R, lam, N->loss.as<float>(),
                         N->dout_f.as<float>(), N->dout_b.as<uint16_t>(), st));
  const uint16_t* wb = N->wbf.as<uint16_t>();
  float* gr = N->grad.as<float>();
  // the upstream gradient of layer l: fp32 (for the bias) and bf16 (for the GEMMs)
  const float* gf = N->dout_f.as<float>();
  const uint16_t* gb = N->dout_b.as<uint16_t>();
  int64_t ldg = N->dout;
  int cur = 0;
  for (int l = 3; l >= 0; --l) {
    const uint16_t* in = l == 0 ? X : N->h[l - 1].as<uint16_t>();
    const int64_t ldin = l == 0 ? N->din : N->width;
    // dW_l[o, i] = sum_b g[b, o] in[b, i]
    GemmArgs gw{};
    gw.A = gb; gw.a_m = 1; gw.a_k = ldg;
    gw.B = in; gw.b_k = ldin; gw.b_n = 1;
    gw.M = N->nout[l]; gw.N = N->nin[l]; gw.K = (int)B;
    gw.Cf = gr + N->oW[l]; gw.ld_cf = N->nin[l];
    HIP_TRY(launch_gemm(gw, st));
    HIP_TRY(launch_colsum(gf, B, N->nout[l], ldg, gr + N->ob[l], st));
    if (l == 0) break;
    // g_{l-1}[b, i] = (sum_o g[b, o] W_l[o, i]) * (h_{l-1}[b, i] > 0)
    GemmArgs gd{};
    gd.A = gb; gd.a_m = ldg; gd.a_k = 1;
    gd.B = wb + N->oW[l]; gd.b_k = N->nin[l]; gd.b_n = 1;
    gd.M = B; gd.N = N->nin[l]; gd.K = N->nout[l];
    gd.mask = N->h[l - 1].as<uint16_t>(); gd.ld_mask = N->width;
    gd.Cf = N->dz_f.as<float>(); gd.ld_cf = N->width;
    gd.Cb = N->dz_b[cur].as<uint16_t>(); gd.ld_cb = N->width;
    HIP_TRY(launch_gemm(gd, st));
    gf = N->dz_f.as<float>();
    gb = N->dz_b[cur].as<uint16_t>();
    ldg = N->width;
    cur ^= 1;
  }
  return FTP_OK;
}

struct ftp_plan {
  int H = 0;
  ftp_options opt{};
  std::vector<double> c, s;
  int device = 0;
  int n_cu = 256;
  std::string arch = "unknown";
  size_t grid_budget = (size_t)8 << 30;   // bytes of NFFT grids per chunk
  // device buffers
  DevBuf alpha, twiddle32, twiddle64, ctab;
  DevBuf pw, py, tile_count, tile_off, cursor, block_sums,
      total, bucket, grids, fft_tab, fft_items, counters, stats_out, rec;
  DevBuf stat_part, stat_ticket;   // statistics kernel: partials per workgroup, ticket per lightcurve
  int64_t stat_slots = 0;          // workgroups of the statistics kernel in this chunk
  int stat_nby = 1;                // the most workgroups of one lightcurve
  int64_t pair_chunk = (int64_t)1 << 20;  // pairs per assemble/root/score round
  int n_band = 0;                          // > 0: band templates for shared-phase calls
  // host staging (kept alive until the uploads completed)
  std::vector<LcInfo> h_lc;
  std::vector<int64_t> h_obs_off, h_freq_off, h_gtb;
  std::vector<int32_t> h_lcb;   // lightcurve of pair b * kLcBlock of the chunk (b = 0..nb), see SolveArgs
  std::vector<FftGridPass> h_fft;
  std::vector<int64_t> h_items;
  std::vector<int64_t> fft_round_tab_off, fft_round_n, fft_round_items;
  std::vector<int> fft_round_el;   // log2 of the largest LDS block (elements) a round's passes use
  // per-chunk tables (lightcurve plans, offsets, FFT passes) packed into one
  // pinned host buffer and sent with one copy; the d_* pointers point into
  // d_stage
  unsigned char* h_stage = nullptr;
  size_t h_stage_cap = 0;
  DevBuf d_stage;
  LcInfo* d_lc = nullptr;
  int64_t *d_obs_off = nullptr, *d_freq_off = nullptr, *d_gtb = nullptr, *d_items = nullptr;
  int32_t* d_lcb = nullptr;
  FftGridPass* d_fft = nullptr;
  hipEvent_t upload_done = nullptr;
  // side stream of the learned / uniform solve: the scoring of the pairs the
  // Newton tier confirmed runs there, beside the Aberth tier (fork after
  // Newton, join before the fallback pairs are scored)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool upload_pending = false;
  size_t stage_sizes[7] = {0, 0, 0, 0, 0, 0, 0};   // piece sizes of the tables last sent (all 0: none)
  ftp_stats last{};
  // stage timing (FTP_FLAG_TIME_STAGES): one event triple per lightcurve chunk
  // (NFFT start, NFFT end, solve end) and one pair per root-kernel launch
  // and one triple per NFFT launch sequence (before the spreading kernel, after
  // it, after the FFT passes)
  std::vector<hipEvent_t> ev, evr, evl, evn;
  int ev_used = 0, evr_used = 0, evl_used = 0, evn_used = 0;
  // learned
  MlpNet net;
  bool mlp_loaded = false;
  // training-set extraction (ftp_learned_dataset): features and real-root labels
  uint16_t* ds_X = nullptr;
  float* ds_roots = nullptr;
  int* ds_nroots = nullptr;
  int ds_R = 0;
  // work lists: Newton -> Aberth (fb_list, count work_ctr[0]) and
  // Aberth -> companion solve (fb2_list, count work_ctr[1]); work_ctr[2..4]
  // are the queue counters of the Newton, Aberth and QR kernels
  DevBuf xfeat, seeds, fb_list, fb2_list, rt_list, work_ctr;
  // launch shapes (waves per compute unit), set by ftp_plan_set_tuning or
  // ftp_autotune
  // default launch shapes: grids far beyond the resident waves for the
  // grid-strided assembly, Newton and scoring kernels (measured on the H
  // sweep's lightcurves: equal or faster at every H, -6 % at H = 11)
  ftp_tuning tune{256, 256, 16, 16, 256, 0, 5};
  DevBuf tune_out;
  // multi-band calls: chi^2_0 of every lightcurve of the batch (device, set
  // for the duration of the call) and the band outputs' scratch
  double* lc_chi2_out = nullptr;
  DevBuf mb_out, mb_chi2;
};

namespace {

int validate_template(int H, const double* c, const double* s) {
  if (!c || !s) return FTP_E_NULL;
  if (H < 1 || H > FTP_MAX_H) return FTP_E_H;
  bool any = false;
  for (int i = 0; i < H; ++i) {
    if (!std::isfinite(c[i]) || !std::isfinite(s[i])) return FTP_E_H;
    if (c[i] != 0.0 || s[i] != 0.0) any = true;
  }
  return any ? FTP_OK : FTP_E_H;
}

int default_msp(int precision) { return precision == FTP_FP64 ? 12 : 7; }

// FFT pass plan: passes (largest stride first) with in-LDS sizes.
// log2 of the elements one FFT workgroup holds in LDS (64 KB)
int fft_max_el(int precision) { return precision == FTP_FP64 ? 12 : 13; }

void fft_plan(int L, int precision, int* npass, int* lp) {
  const int last = precision == FTP_FP64 ? 11 : 12;   // largest single pass (twiddle table)
  const int wide = fft_max_el(precision) - 4;         // earlier passes: 16 columns per workgroup
  if (L <= last) { *npass = 1; lp[0] = L; return; }
  const int rest = L - last;
  const int npre = (rest + wide - 1) / wide;
  int k = 0;
  for (int p = 0; p < npre; ++p) {
    const int take = rest / npre + (p < rest % npre ? 1 : 0);
    lp[k++] = take;
  }
  lp[k++] = last;
  *npass = k;
}

// Returns the next timing event (creating it on demand), or nullptr.
hipEvent_t next_event_in(ftp_plan* P, std::vector<hipEvent_t>& pool, int& used) {
  if (!(P->opt.flags & FTP_FLAG_TIME_STAGES)) return nullptr;
  if (used == (int)pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[used++];
}
hipEvent_t next_event(ftp_plan* P) { return next_event_in(P, P->ev, P->ev_used); }
hipEvent_t next_root_event(ftp_plan* P) { return next_event_in(P, P->evr, P->evr_used); }
hipEvent_t next_learn_event(ftp_plan* P) { return next_event_in(P, P->evl, P->evl_used); }
hipEvent_t next_nfft_event(ftp_plan* P) { return next_event_in(P, P->evn, P->evn_used); }

int wait_uploads(ftp_plan* P) {
  if (P->upload_pending) {
    HIP_TRY(hipEventSynchronize(P->upload_done));
    P->upload_pending = false;
  }
  return FTP_OK;
}

int validate_scalars(double df, int64_t n_f, int64_t n_obs) {
  if (n_obs < 3) return FTP_E_NOBS;
  if (!(std::isfinite(df) && df > 0.0)) return FTP_E_DF;
  if (n_f < 1) return FTP_E_NF;
  // grid modes 2 H n_f must fit the int64 index math and the 2^30 grid cap
  if (n_f > (int64_t)1 << 26) return FTP_E_SIZE;
  if (n_obs > (int64_t)1 << 29) return FTP_E_SIZE;
  return FTP_OK;
}

struct Chunk {
  int64_t lc0, lc1;   // [lc0, lc1)
};

// Fill LcInfo plan fields for lightcurves [lc0, lc1), return grid elements.
int plan_chunk(ftp_plan* P, int64_t lc0, int64_t lc1, const int64_t* obs_off, const double* df,
               const int64_t* freq_off, int64_t* n_grid_elems, int64_t* n_tiles) {
  const int H = P->H;
  const double R = P->opt.nfft_R > 0 ? P->opt.nfft_R : 2.0;
  const int msp = P->opt.nfft_msp > 0 ? P->opt.nfft_msp : default_msp(P->opt.precision);
  const int64_t n = lc1 - lc0;
  P->h_lc.assign(n, LcInfo{});
  P->h_obs_off.assign(n + 1, 0);
  P->h_freq_off.assign(n + 1, 0);
  P->h_gtb.assign(2 * n + 1, 0);
  int64_t goff = 0, tbase = 0, stat_slots = 0;
  P->stat_nby = 1;
  for (int64_t b = 0; b < n; ++b) {
    LcInfo& L = P->h_lc[b];
    const int64_t gb = lc0 + b;
    L.obs_off = obs_off[gb] - obs_off[lc0];
    L.n_obs = obs_off[gb + 1] - obs_off[gb];
    L.freq_off = freq_off[gb] - freq_off[lc0];
    L.n_f = freq_off[gb + 1] - freq_off[gb];
    L.df = df[gb];
    L.msp = msp;
    // the statistics kernel's workgroups depend on n_obs alone, so a lightcurve
    // is reduced in the same order alone and inside a batch
    L.stat_nb = (int)std::min<int64_t>(kStatMaxBlocks, std::max<int64_t>(1, (L.n_obs + 511) / 512));
    L.stat_off = stat_slots;
    stat_slots += L.stat_nb;
    P->stat_nby = std::max(P->stat_nby, L.stat_nb);
    P->h_obs_off[b] = L.obs_off;
    P->h_freq_off[b] = L.freq_off;
    for (int g = 0; g < 2; ++g) {
      const int64_t mmax = g == 0 ? 2LL * H * L.n_f : (int64_t)H * L.n_f;
      const int64_t M = mmax + 1;
      int log2n = ilog2_ceil((int64_t)std::ceil(R * (double)M));
      log2n = std::max(log2n, 12);
      if (log2n > 30) return FTP_E_SIZE;
      const int64_t nn = 1LL << log2n;
      const double Reff = (double)nn / (double)M;
      L.log2n[g] = log2n;
      L.mc[g] = mmax / 2;
      L.beta[g] = M_PI * (Reff - 0.5) / (msp * Reff);
      L.dec_a[g] = std::sqrt(L.beta[g] / M_PI);
      L.dec_b[g] = M_PI * M_PI / ((double)nn * (double)nn * L.beta[g]);
      fft_plan(log2n, P->opt.precision, &L.npass[g], L.lp[g]);
      L.grid_off[g] = goff;
      goff += nn;
      L.tile_base[g] = tbase;
      P->h_gtb[2 * b + g] = tbase;
      tbase += nn / kTileCells;
    }
  }
  P->stat_slots = stat_slots;
  P->h_obs_off[n] = obs_off[lc1] - obs_off[lc0];
  P->h_freq_off[n] = freq_off[lc1] - freq_off[lc0];
  P->h_gtb[2 * n] = tbase;
  {
    // lightcurve of every kLcBlock-th pair (and of the last): a pair's
    // lightcurve lies between its block's two entries
    const int64_t np_chunk = P->h_freq_off[n];
    const int64_t nb = (np_chunk + kLcBlock - 1) / kLcBlock;
    P->h_lcb.resize((size_t)nb + 1);
    int64_t lc = 0;
    for (int64_t b = 0; b <= nb; ++b) {
      const int64_t pr = std::min<int64_t>(b * kLcBlock, std::max<int64_t>(np_chunk - 1, 0));
      while (lc + 1 < n && P->h_freq_off[lc + 1] <= pr) ++lc;
      P->h_lcb[b] = (int32_t)lc;
    }
  }
  *n_grid_elems = goff;
  *n_tiles = tbase;
  return FTP_OK;
}

template <typename R>
int run_nfft(ftp_plan* P, int64_t n_lc, int64_t n_pts, int64_t n_grid, int64_t n_tiles, int shared_bands, const double* t,
             const double* y, const double* sigma, hipStream_t st) {
  using C = typename Cplx<R>::T;
  int rc;
  if ((rc = P->pw.ensure(sizeof(PointRec<R>) * std::max<int64_t>(n_pts, 1)))) return rc;
  if ((rc = P->py.ensure(sizeof(PointRec<R>) * std::max<int64_t>(n_pts, 1)))) return rc;
  if ((rc = P->tile_count.ensure(sizeof(unsigned) * n_tiles))) return rc;
  if ((rc = P->cursor.ensure(sizeof(unsigned) * n_tiles))) return rc;
  if ((rc = P->tile_off.ensure(sizeof(int64_t) * (n_tiles + 1)))) return rc;
  const int64_t nsb = (n_tiles + 1023) / 1024;
  if ((rc = P->block_sums.ensure(sizeof(int64_t) * (nsb + 1)))) return rc;
  if ((rc = P->total.ensure(sizeof(int64_t)))) return rc;
  if ((rc = P->bucket.ensure(sizeof(int) * std::max<int64_t>(4 * n_pts, 1)))) return rc;
  if ((rc = P->grids.ensure(sizeof(C) * n_grid))) return rc;
  LcInfo* dl = P->d_lc;
  // statistics: stat_nb workgroups per lightcurve, combined by the last of
  // them; the tickets start at 0 and every call leaves them at 0
  if ((rc = P->stat_part.ensure(sizeof(double) * kStatVals * P->stat_slots))) return rc;
  {
    const size_t cap0 = P->stat_ticket.cap;
    if ((rc = P->stat_ticket.ensure(sizeof(unsigned) * n_lc))) return rc;
    if (P->stat_ticket.cap != cap0)
      HIP_TRY(launch_zero_u32(P->stat_ticket.as<unsigned>(), (int64_t)(P->stat_ticket.cap / sizeof(unsigned)), st));
  }
  // (it also clears the tile histogram and the binning cursors)
  hipLaunchKernelGGL(k_prep_stats, dim3((unsigned)n_lc, (unsigned)P->stat_nby), dim3(kStatThreads), 0, st, dl, t, y,
                     sigma, P->stat_part.as<double>(), P->stat_ticket.as<unsigned>(), P->tile_count.as<unsigned>(),
                     P->cursor.as<unsigned>(), n_tiles);
  if (shared_bands > 0)
    hipLaunchKernelGGL(k_sp_combine, dim3(1), dim3(64), 0, st, dl, shared_bands, P->alpha.as<double2>(), P->H);
  const unsigned pblocks = (unsigned)((n_pts + 255) / 256);
  hipLaunchKernelGGL(k_prep_points<R>, dim3(pblocks), dim3(256), 0, st, dl, n_lc,
                     P->d_obs_off, n_pts, t, y, sigma, P->pw.as<PointRec<R>>(),
                     P->py.as<PointRec<R>>(), P->tile_count.as<unsigned>());
  if (n_tiles <= kScanSingleMax) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, P->tile_count.as<unsigned>(), n_tiles,
                       P->tile_off.as<int64_t>(), P->total.as<int64_t>());
  } else {
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nsb), dim3(256), 0, st, P->tile_count.as<unsigned>(),
                       n_tiles, P->tile_off.as<int64_t>(), P->block_sums.as<int64_t>());
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, st, P->block_sums.as<int64_t>(), nsb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nsb), dim3(256), 0, st, P->tile_off.as<int64_t>(), n_tiles,
                       P->block_sums.as<int64_t>(), P->tile_count.as<unsigned>(), P->total.as<int64_t>());
  }
  hipLaunchKernelGGL(k_bin_fill<R>, dim3(pblocks), dim3(256), 0, st, dl, n_lc, P->d_obs_off,
                     n_pts, P->pw.as<PointRec<R>>(), P->py.as<PointRec<R>>(), P->tile_off.as<int64_t>(),
                     P->cursor.as<unsigned>(), P->bucket.as<int>());
  hipEvent_t s0 = next_nfft_event(P);
  if (s0) HIP_TRY(hipEventRecord(s0, st));
  hipLaunchKernelGGL(k_spread<R>, dim3((unsigned)n_tiles), dim3(256), 0, st, dl, 2 * n_lc,
                     P->d_gtb, P->pw.as<PointRec<R>>(), P->py.as<PointRec<R>>(),
                     P->tile_off.as<int64_t>(), P->bucket.as<int>(), P->grids.as<C>());
  hipEvent_t s1 = next_nfft_event(P);
  if (s1) HIP_TRY(hipEventRecord(s1, st));
  const C* tw = reinterpret_cast<const C*>(P->opt.precision == FTP_FP64 ? P->twiddle64.p : P->twiddle32.p);
  int64_t item_base = 0;
  for (size_t r = 0; r < P->fft_round_n.size(); ++r) {
    // LDS for the round's largest block only (more workgroups per CU)
    hipLaunchKernelGGL(k_fft_pass<R>, dim3((unsigned)P->fft_round_items[r]), dim3(256),
                       sizeof(C) << P->fft_round_el[r], st,
                       P->d_fft + P->fft_round_tab_off[r], P->fft_round_n[r], P->d_items + item_base, tw,
                       P->grids.as<C>(), P->tile_off.as<int64_t>());
    item_base += P->fft_round_n[r] + 1;
  }
  hipEvent_t s2 = next_nfft_event(P);
  if (s2) HIP_TRY(hipEventRecord(s2, st));
  HIP_TRY(hipGetLastError());
  return FTP_OK;
}

// FFT passes of the chunk's grids (host): per round, one FftGridPass per grid
// that still has a pass, and the item offsets of each round.
void build_fft_tables(ftp_plan* P) {
  int max_pass = 0;
  for (const LcInfo& L : P->h_lc) max_pass = std::max({max_pass, L.npass[0], L.npass[1]});
  std::vector<FftGridPass>& tab = P->h_fft;
  std::vector<int64_t>& items = P->h_items;
  tab.clear();
  items.clear();
  P->fft_round_tab_off.clear();
  P->fft_round_n.clear();
  P->fft_round_items.clear();
  P->fft_round_el.clear();
  for (int r = 0; r < max_pass; ++r) {
    P->fft_round_tab_off.push_back((int64_t)tab.size());
    int64_t it = 0;
    int64_t cnt = 0;
    int el = 0;
    for (const LcInfo& L : P->h_lc) {
      for (int g = 0; g < 2; ++g) {
        if (L.npass[g] <= r) continue;
        FftGridPass fp{};
        fp.grid_off = L.grid_off[g];
        fp.item_begin = it;
        fp.tile_base = r == 0 ? L.tile_base[g] : -1;
        fp.log2n = L.log2n[g];
        fp.lp = L.lp[g][r];
        int consumed = 0;
        for (int q = 0; q <= r; ++q) consumed += L.lp[g][q];
        fp.ls = fp.log2n - consumed;
        const int maxel = fft_max_el(P->opt.precision);
        fp.lcols = std::min(fp.ls, std::min(4, maxel - fp.lp));
        el = std::max(el, fp.lp + fp.lcols);
        tab.push_back(fp);
        it += 1LL << (fp.log2n - fp.lp - fp.lcols);
        ++cnt;
      }
    }
    P->fft_round_n.push_back(cnt);
    P->fft_round_items.push_back(it);
    P->fft_round_el.push_back(el);
  }
  // item_begin arrays per round, laid out after each other (with sentinel)
  for (int r = 0; r < max_pass; ++r) {
    for (int64_t q = 0; q < P->fft_round_n[r]; ++q) items.push_back(tab[P->fft_round_tab_off[r] + q].item_begin);
    items.push_back(P->fft_round_items[r]);
  }
}

// Sends the chunk's tables (and, with_fft, its FFT passes) in one copy from
// pinned staging.  The staging is reused once this copy has completed
// (upload_done, waited for by the next call).
int upload_tables(ftp_plan* P, int64_t n_lc, hipStream_t st, bool with_fft) {
  int rc;
  if ((rc = wait_uploads(P))) return rc;
  if (with_fft) build_fft_tables(P);
  else {
    P->h_fft.clear();
    P->h_items.clear();
  }
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t s_lc = sizeof(LcInfo) * n_lc, s_off = sizeof(int64_t) * (n_lc + 1),
               s_gtb = sizeof(int64_t) * (2 * n_lc + 1), s_fft = sizeof(FftGridPass) * P->h_fft.size(),
               s_it = sizeof(int64_t) * P->h_items.size(), s_lcb = sizeof(int32_t) * P->h_lcb.size();
  const size_t o_lc = 0, o_obs = al(o_lc + s_lc), o_freq = al(o_obs + s_off), o_gtb = al(o_freq + s_off),
               o_fft = al(o_gtb + s_gtb), o_it = al(o_fft + s_fft), o_lcb = al(o_it + s_it),
               total = al(o_lcb + s_lcb);
  if (total > P->h_stage_cap) {
    for (int k = 0; k < 7; ++k) P->stage_sizes[k] = 0;
    if (P->h_stage) HIP_TRY(hipHostFree(P->h_stage));
    P->h_stage = nullptr;
    P->h_stage_cap = 0;
    HIP_TRY(hipHostMalloc((void**)&P->h_stage, total, hipHostMallocDefault));
    P->h_stage_cap = total;
  }
  unsigned char* h = P->h_stage;
  // the staging still holds the tables last sent, and the device copy is
  // complete (waited for above); the kernels rewrite only the fields the
  // device fills, which the host leaves 0. Tables equal to those need no copy.
  const size_t sizes[7] = {s_lc, s_off, s_off, s_gtb, s_fft, s_it, s_lcb};
  const void* src[7] = {P->h_lc.data(), P->h_obs_off.data(), P->h_freq_off.data(), P->h_gtb.data(),
                        P->h_fft.data(), P->h_items.data(), P->h_lcb.data()};
  const size_t offs[7] = {o_lc, o_obs, o_freq, o_gtb, o_fft, o_it, o_lcb};
  bool same = P->d_stage.p != nullptr && P->d_stage.cap >= total;
  for (int k = 0; k < 7 && same; ++k)
    same = sizes[k] == P->stage_sizes[k] && (sizes[k] == 0 || std::memcmp(h + offs[k], src[k], sizes[k]) == 0);
  if (!same) {
    for (int k = 0; k < 7; ++k) P->stage_sizes[k] = 0;
    for (int k = 0; k < 7; ++k)
      if (sizes[k]) std::memcpy(h + offs[k], src[k], sizes[k]);
    if ((rc = P->d_stage.ensure(total))) return rc;
    HIP_TRY(hipMemcpyAsync(P->d_stage.p, h, total, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(P->upload_done, st));
    P->upload_pending = true;
    for (int k = 0; k < 7; ++k) P->stage_sizes[k] = sizes[k];
  }
  unsigned char* d = P->d_stage.as<unsigned char>();
  P->d_lc = reinterpret_cast<LcInfo*>(d + o_lc);
  P->d_obs_off = reinterpret_cast<int64_t*>(d + o_obs);
  P->d_freq_off = reinterpret_cast<int64_t*>(d + o_freq);
  P->d_gtb = reinterpret_cast<int64_t*>(d + o_gtb);
  P->d_fft = reinterpret_cast<FftGridPass*>(d + o_fft);
  P->d_items = reinterpret_cast<int64_t*>(d + o_it);
  P->d_lcb = s_lcb ? reinterpret_cast<int32_t*>(d + o_lcb) : nullptr;
  return FTP_OK;
}

// Grid of a per-frequency kernel: the option override, else the tuned waves
// per compute unit; never more waves than pairs.
int64_t grid_waves(const ftp_plan* P, int wpc, int64_t np) {
  const int64_t w = P->opt.solve_waves > 0 ? (int64_t)P->opt.solve_waves : (int64_t)wpc * P->n_cu;
  return std::max<int64_t>(1, std::min<int64_t>(w, np));
}

// Per-frequency stage over pair chunks: assemble -> roots -> score.  Roots:
// companion QR (plain); network features -> MLP -> Newton + Sturm -> Aberth
// on the unconfirmed pairs -> companion QR on what Aberth leaves (learned,
// and the uniform-start ablation without the network); Aberth on every pair
// -> companion QR on what it leaves (Aberth).  The root kernels take their
// pairs from queue counters.
// Scratch of the per-frequency stage: records and work lists for chunks of
// up to `chunk` pairs, and the 8 work counters.
struct SolveBufs {
  double* rec;
  unsigned* ctr;
  int64_t* fb_list;          // first Newton round -> second round
  int64_t* fb2_list;         // Aberth tier -> companion solve
  int64_t* rt_list;          // second Newton round -> Aberth tier
  int64_t chunk;
  SolveCounters* counters;   // statistics copies (nullptr: none kept)
  bool timing;               // stage events (FTP_FLAG_TIME_STAGES)
};

// The plan's own scratch for n_pairs pairs (grown on demand).
int solve_bufs_plan(ftp_plan* P, int64_t n_pairs, SolveBufs* B) {
  const RecLayout RL(P->H);
  const int64_t chunk = std::min<int64_t>(n_pairs, P->pair_chunk);
  int rc;
  if ((rc = P->rec.ensure(sizeof(double) * (size_t)chunk * RL.stride))) return rc;
  if ((rc = P->work_ctr.ensure(8 * sizeof(unsigned)))) return rc;
  const int solver = P->ds_X != nullptr ? FTP_SOLVER_PLAIN : P->opt.solver;
  if (solver != FTP_SOLVER_PLAIN) {
    if ((rc = P->fb_list.ensure(sizeof(int64_t) * chunk))) return rc;
    if ((rc = P->fb2_list.ensure(sizeof(int64_t) * chunk))) return rc;
    if ((rc = P->rt_list.ensure(sizeof(int64_t) * chunk))) return rc;
    if (solver == FTP_SOLVER_LEARNED) {
      if ((rc = P->xfeat.ensure(sizeof(uint16_t) * chunk * P->net.din))) return rc;
      if ((rc = P->seeds.ensure(sizeof(float) * chunk * P->net.dout))) return rc;
      if ((rc = P->net.ensure_batch(chunk))) return rc;
    }
  }
  B->rec = P->rec.as<double>();
  B->ctr = P->work_ctr.as<unsigned>();
  B->fb_list = P->fb_list.as<int64_t>();
  B->fb2_list = P->fb2_list.as<int64_t>();
  B->rt_list = P->rt_list.as<int64_t>();
  B->chunk = chunk;
  B->counters = P->counters.as<SolveCounters>();
  B->timing = (P->opt.flags & FTP_FLAG_TIME_STAGES) != 0;
  return FTP_OK;
}

int run_solve_with(ftp_plan* P, const SolveArgs& a0, int64_t n_pairs, const SolveBufs& B, hipStream_t st);

int run_solve(ftp_plan* P, const SolveArgs& a, int64_t n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return FTP_OK;
  SolveBufs B;
  int rc;
  if ((rc = solve_bufs_plan(P, n_pairs, &B))) return rc;
  return run_solve_with(P, a, n_pairs, B, st);
}

// The per-frequency stage over n_pairs pairs in chunks of B.chunk, with the
// scratch in B (the learned solver also uses the plan's network buffers).
int run_solve_with(ftp_plan* P, const SolveArgs& a0, int64_t n_pairs, const SolveBufs& B, hipStream_t st) {
  if (n_pairs <= 0) return FTP_OK;
  const RecLayout RL(P->H);
  const int64_t chunk = B.chunk;
  int rc;
  SolveArgs a = a0;
  a.counters = B.counters;
  double* rec = B.rec;
  unsigned* ctr = B.ctr;
  const bool dataset = P->ds_X != nullptr;
  const int solver = dataset ? FTP_SOLVER_PLAIN : P->opt.solver;
  auto root_ev = [&]() -> hipEvent_t { return B.timing ? next_root_event(P) : nullptr; };
  auto learn_ev = [&]() -> hipEvent_t { return B.timing ? next_learn_event(P) : nullptr; };
  const ftp_tuning& T = P->tune;
  // scoring of the Newton-root pairs four per wavefront, on the side stream
  const bool overlap_score =
      !dataset && (solver == FTP_SOLVER_LEARNED || solver == FTP_SOLVER_UNIFORM) && 6 * P->H - 2 < 64;
  // learned solver with a fusable network: features in rows of dinp bf16
  // (zero padded), then one kernel for the four layers
  const bool fused = solver == FTP_SOLVER_LEARNED && P->tune.mlp_fused && P->net.dense &&
                     mlp_fused_ok(P->net.nin, P->net.nout);
  const int dinp = (P->net.din + 31) & ~31;
  if ((fused || P->net.dense) && (rc = P->xfeat.ensure(sizeof(uint16_t) * chunk * dinp))) return rc;
  for (int64_t p0 = 0; p0 < n_pairs; p0 += chunk) {
    const int64_t np = std::min<int64_t>(chunk, n_pairs - p0);
    const int w_asm = (int)grid_waves(P, T.assemble_wpc, np);
    const int w_qr = (int)grid_waves(P, T.qr_wpc, np);
    const int w_nt = (int)grid_waves(P, T.newton_wpc, np);
    const int w_ab = (int)grid_waves(P, T.aberth_wpc, np);
    const int w_sc = (int)grid_waves(P, T.score_wpc, np);
    {
      // the assembly also clears the chunk's counters (no kernel of the
      // previous chunk reads them once its scoring has run)
      SolveArgs aa = a;
      aa.clear8 = ctr;
      HIP_TRY(launch_assemble(P->opt.precision, aa, rec, p0, np, w_asm, st));
    }
    hipEvent_t r0 = root_ev();
    if (r0) HIP_TRY(hipEventRecord(r0, st));
    if (solver == FTP_SOLVER_PLAIN) {
      HIP_TRY(launch_qr(P->H, rec, RL.stride, np, nullptr, nullptr, B.counters, ctr + 4, w_qr,
                        st));
    } else {
      // the network's seeds: for every pair's first round (FTP_FLAG_SEEDS_ALL),
      // else for the pairs the first round leaves (list and its device count)
      // done (nullable): an event recorded once the seeds are written
      auto run_network = [&](const int64_t* list, const unsigned* count, hipEvent_t done) -> int {
        MlpNet& N = P->net;
        if (fused) {
          HIP_TRY(launch_features(rec, P->H, np, P->xfeat.as<uint16_t>(), dinp, w_asm, st, list, count));
          FusedMlpArgs fa{};
          fa.X = P->xfeat.as<uint16_t>();
          fa.np = np;
          fa.wi = N.winf.as<uint16_t>();
          fa.w32 = N.w32.as<float>();
          for (int l = 0; l < 4; ++l) {
            fa.oWi[l] = N.oWi[l];
            fa.ob[l] = N.ob[l];
            fa.kp[l] = N.kp[l];
            fa.nout[l] = N.nout[l];
          }
          fa.out = P->seeds.as<float>();
          fa.np_dev = count;
          HIP_TRY(launch_mlp_fused(fa, st, 2 * P->n_cu, done));
          return FTP_OK;
        }
        // (the layer-by-layer forms run over all np rows; rows past the list
        // hold stale features and their outputs are not read)
        int r2;
        if (N.dense) {
          HIP_TRY(launch_features(rec, P->H, np, P->xfeat.as<uint16_t>(), dinp, w_asm, st, list, count));
          r2 = mlp_forward_dense(&N, P->xfeat.as<uint16_t>(), dinp, np, P->seeds.as<float>(), st);
        } else {
          HIP_TRY(launch_features(rec, P->H, np, P->xfeat.as<uint16_t>(), N.din, w_asm, st, list, count));
          r2 = mlp_forward(&N, P->xfeat.as<uint16_t>(), np, P->seeds.as<float>(), st);
        }
        if (!r2 && done) HIP_TRY(hipEventRecord(done, st));
        return r2;
      };
      const bool seeds_all = solver == FTP_SOLVER_LEARNED && (P->opt.flags & FTP_FLAG_SEEDS_ALL);
      const bool net_list = solver == FTP_SOLVER_LEARNED && !seeds_all;
      const float* seeds = nullptr;
      if (seeds_all) {
        if ((rc = run_network(nullptr, nullptr, nullptr))) return rc;
        seeds = P->seeds.as<float>();
      }
      hipEvent_t ra = learn_ev();
      if (ra) HIP_TRY(hipEventRecord(ra, st));
      if (solver != FTP_SOLVER_ABERTH) {
        LearnArgs L{};
        L.rec = rec;
        L.np = np;
        L.seeds_out = seeds;
        L.fb_list = B.fb_list;
        L.fb_count = ctr;
        L.flags = ((P->opt.flags & FTP_FLAG_FORCE_FALLBACK) ? 1u : 0u) | ((P->opt.flags & FTP_FLAG_2H_STARTS) ? 2u : 0u);
        L.queue = nullptr;   // uniform work per pair: grid striding (a queue costs more than it balances)
        // with the side stream, the Newton kernel and the side scoring launch
        // record the fork and join events themselves: the scoring of the
        // Newton-root pairs is the longest branch after the fork, so it starts
        // as soon as the first round ends beside the later tiers (uniform
        // solver); with the network on the first round's list it starts after
        // the second round instead, so that the network's large workgroups
        // and the round do not wait for CU room behind the scoring's
        // wavefronts (measured: learned -15 us, uniform +11 us that way)
        HIP_TRY(launch_newton_sturm(a, L, w_nt, T.newton_occ, st, (overlap_score && !net_list) ? P->fork_ev : nullptr));
      }
      hipEvent_t rb = learn_ev();
      if (rb) HIP_TRY(hipEventRecord(rb, st));
      // second Newton round on what the first left: the network's seeds for
      // the learned solver (unless every pair had them already), evenly spaced
      // starts otherwise; what it leaves goes to the Aberth tier
      if (net_list) {
        if ((rc = run_network(B.fb_list, ctr, nullptr))) return rc;
      }
      // the Newton-root pairs are final now: score them on the side stream
      // while the later tiers run on this one
      auto fork_score = [&]() -> int {
        SolveArgs as = a;
        as.newton_cands = true;
        HIP_TRY(hipStreamWaitEvent(P->side, P->fork_ev, 0));
        HIP_TRY(launch_score_newton(as, rec, p0, np, w_sc, P->side, P->join_ev));
        return FTP_OK;
      };
      if (solver != FTP_SOLVER_ABERTH && overlap_score && !net_list) {
        if ((rc = fork_score())) return rc;
      }
      hipEvent_t rr = learn_ev();
      if (rr) HIP_TRY(hipEventRecord(rr, st));
      if (solver != FTP_SOLVER_ABERTH) {
        RetryArgs RA{};
        RA.rec = rec;
        RA.H = P->H;
        RA.list = B.fb_list;
        RA.count = ctr;
        RA.seeds = (solver == FTP_SOLVER_LEARNED && !seeds_all) ? P->seeds.as<float>() : nullptr;
        RA.out_list = B.rt_list;
        RA.out_count = ctr + 5;
        RA.counters = B.counters;
        // (one wavefront per listed frequency: a grid at least as long as the
        // list gives no wavefront a second one)
        HIP_TRY(launch_newton_retry(RA, (int)grid_waves(P, 64, np), st));
      }
      if (solver != FTP_SOLVER_ABERTH && overlap_score && net_list) {
        HIP_TRY(hipEventRecord(P->fork_ev, st));
        if ((rc = fork_score())) return rc;
      }
      hipEvent_t rt = learn_ev();
      if (rt) HIP_TRY(hipEventRecord(rt, st));
      AberthArgs A{};
      A.rec = rec;
      A.np = np;
      A.list = solver == FTP_SOLVER_ABERTH ? nullptr : B.rt_list;
      A.count = ctr + 5;
      A.qr_list = B.fb2_list;
      A.qr_count = ctr + 1;
      A.counters = B.counters;
      A.H = P->H;
      A.mark = 2.0;
      A.flags = (P->opt.flags & FTP_FLAG_FORCE_FALLBACK) ? 1u : 0u;
      A.queue = ctr + 3;
      HIP_TRY(launch_aberth(A, w_ab, st));
      hipEvent_t rc2 = learn_ev();
      if (rc2) HIP_TRY(hipEventRecord(rc2, st));
      // what the Aberth tier leaves is usually nothing or a few frequencies:
      // a launch of one wave per CU serves it through the queue.  Above
      // D = 64 (or with the forced fallback) the Sturm count is refused on
      // most frequencies and the list holds most of them: the plain solve's
      // launch shape
      const bool big_list = 6 * P->H - 2 > 64 || (P->opt.flags & FTP_FLAG_FORCE_FALLBACK);
      HIP_TRY(launch_qr(P->H, rec, RL.stride, np, B.fb2_list, ctr + 1, B.counters, ctr + 4,
                        big_list ? w_qr : std::min(w_qr, (int)grid_waves(P, 1, np)), st));
    }
    hipEvent_t r1 = root_ev();
    if (r1) HIP_TRY(hipEventRecord(r1, st));
    if (dataset) {
      HIP_TRY(launch_features(rec, P->H, np, P->ds_X + p0 * (int64_t)(2 * (6 * P->H - 1)), 2 * (6 * P->H - 1),
                              w_asm, st));
      HIP_TRY(launch_labels(rec, P->H, np, P->ds_roots + p0 * (int64_t)P->ds_R, P->ds_nroots + p0, P->ds_R, w_asm,
                            st));
    } else {
      SolveArgs as = a;
      as.newton_cands = solver == FTP_SOLVER_LEARNED || solver == FTP_SOLVER_UNIFORM;
      if (overlap_score) {
        // the fallback list here, while the Newton-root pairs (M_FALLBACK = 0,
        // a disjoint set: neither kernel reads what the other writes) may
        // still be scored on the side stream; the join then orders the side
        // stream's outputs before whatever follows on this one (the next
        // chunk's assembly rewrites the records)
        HIP_TRY(launch_score(as, rec, p0, np, std::min(w_sc, (int)grid_waves(P, 16, np)), st,
                             B.fb_list, ctr));
        HIP_TRY(hipStreamWaitEvent(st, P->join_ev, 0));
      } else {
        HIP_TRY(launch_score(as, rec, p0, np, w_sc, st));
      }
    }
  }
  return FTP_OK;
}

SolveArgs base_args(ftp_plan* P, int64_t n_lc, int64_t n_pairs) {
  SolveArgs a{};
  a.lcs = P->d_lc;
  a.n_lc = n_lc;
  a.freq_off = P->d_freq_off;
  a.lc_block = n_lc > 1 ? P->d_lcb : nullptr;
  a.total = n_pairs;
  a.grids = P->grids.p;
  a.alpha = P->alpha.as<double2>();
  a.ctab = P->ctab.as<double>();
  a.H = P->H;
  a.flags = (int)P->opt.flags;
  a.mm_tau = P->opt.precision == FTP_FP64 ? 1e-9 : 1e-5;
  a.counters = P->counters.as<SolveCounters>();
  return a;
}

template <typename R>
int run_chunk(ftp_plan* P, int64_t lc0, int64_t lc1, const int64_t* obs_off, const double* df,
              const int64_t* freq_off, const double* t, const double* y, const double* sigma, double* power,
              double* phase, double* amp, double* offset, uint8_t* status, double* sums_out, hipStream_t st) {
  int rc;
  if ((rc = wait_uploads(P))) return rc;
  int64_t n_grid = 0, n_tiles = 0;
  if ((rc = plan_chunk(P, lc0, lc1, obs_off, df, freq_off, &n_grid, &n_tiles))) return rc;
  const int64_t n_lc = lc1 - lc0;
  if ((rc = upload_tables(P, n_lc, st, true))) return rc;
  const int64_t o0 = obs_off[lc0], n_pts = obs_off[lc1] - o0;
  const int64_t f0 = freq_off[lc0], n_pairs = freq_off[lc1] - f0;
  hipEvent_t e0 = next_event(P);
  if (e0) HIP_TRY(hipEventRecord(e0, st));
  if ((rc = run_nfft<R>(P, n_lc, n_pts, n_grid, n_tiles, 0, t + o0, y + o0, sigma + o0, st))) return rc;
  hipEvent_t e1 = next_event(P);
  if (e1) HIP_TRY(hipEventRecord(e1, st));
  if (P->lc_chi2_out) HIP_TRY(launch_lc_chi2(P->d_lc, n_lc, P->lc_chi2_out + lc0, st));
  SolveArgs a = base_args(P, n_lc, n_pairs);
  if (sums_out) {
    const int64_t blocks = std::min<int64_t>(n_pairs, 65536);
    HIP_TRY(launch_gather_sums(P->opt.precision, a, sums_out, (int)blocks, st));
  } else {
    a.power = power + f0;
    a.phase = phase + f0;
    a.amp = amp + f0;
    a.offset = offset + f0;
    a.status = status ? status + f0 : nullptr;
    if ((rc = run_solve(P, a, n_pairs, st))) return rc;
  }
  hipEvent_t e2 = next_event(P);
  if (e2) HIP_TRY(hipEventRecord(e2, st));
  return FTP_OK;
}

int run_batch(ftp_plan* P, int64_t n_lc, const int64_t* obs_off, const double* t, const double* y,
              const double* sigma, const double* df, const int64_t* freq_off, double* power, double* phase,
              double* amp, double* offset, uint8_t* status, double* sums_out, hipStream_t st) {
  int rc;
  if (P->opt.solver == FTP_SOLVER_LEARNED && !P->mlp_loaded && !P->ds_X) return FTP_E_NO_MODEL;
  if (P->n_band) return FTP_E_OPTION;   // band templates: shared-phase calls only
  // chunk by grid memory
  const size_t esz = P->opt.precision == FTP_FP64 ? 16 : 8;
  int64_t lc0 = 0;
  const double R = P->opt.nfft_R > 0 ? P->opt.nfft_R : 2.0;
  while (lc0 < n_lc) {
    int64_t lc1 = lc0;
    size_t bytes = 0;
    while (lc1 < n_lc) {
      const int64_t nf = freq_off[lc1 + 1] - freq_off[lc1];
      size_t b = 0;
      for (int g = 0; g < 2; ++g) {
        const int64_t M = (g == 0 ? 2LL * P->H * nf : (int64_t)P->H * nf) + 1;
        b += ((size_t)1 << std::max(12, ilog2_ceil((int64_t)std::ceil(R * (double)M)))) * esz;
      }
      if (lc1 > lc0 && bytes + b > P->grid_budget) break;
      bytes += b;
      ++lc1;
    }
    if (P->opt.precision == FTP_FP64)
      rc = run_chunk<double>(P, lc0, lc1, obs_off, df, freq_off, t, y, sigma, power, phase, amp, offset, status,
                             sums_out, st);
    else
      rc = run_chunk<float>(P, lc0, lc1, obs_off, df, freq_off, t, y, sigma, power, phase, amp, offset, status,
                            sums_out, st);
    if (rc) return rc;
    lc0 = lc1;
  }
  P->last.n_pairs += (uint64_t)freq_off[n_lc];
  return FTP_OK;
}

bool tuning_valid(const ftp_tuning& t) {
  const int v[5] = {t.assemble_wpc, t.newton_wpc, t.aberth_wpc, t.qr_wpc, t.score_wpc};
  for (int x : v)
    if (x < 1 || x > 256) return false;
  return (t.mlp_fused == 0 || t.mlp_fused == 1) && t.newton_occ >= 4 && t.newton_occ <= 6;
}

bool key_valid(const char* key) {
  if (!key || !*key) return false;
  for (const char* c = key; *c; ++c)
    if (std::isspace((unsigned char)*c)) return false;
  return true;
}

// Device time of one periodogram call (ms) on stream st.
int time_call(ftp_plan* P, const double* t, const double* y, const double* sigma, int64_t n_obs, double df,
              int64_t n_f, hipStream_t st, float* ms) {
  double* out = P->tune_out.as<double>();
  uint8_t* status = reinterpret_cast<uint8_t*>(out + 4 * n_f);
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  const int64_t obs_off[2] = {0, n_obs};
  const int64_t freq_off[2] = {0, n_f};
  HIP_TRY(hipEventRecord(a, st));
  int rc = run_batch(P, 1, obs_off, t, y, sigma, &df, freq_off, out, out + n_f, out + 2 * n_f, out + 3 * n_f,
                     status, nullptr, st);
  if (rc == FTP_OK) {
    HIP_TRY(hipEventRecord(b, st));
    HIP_TRY(hipEventSynchronize(b));
    HIP_TRY(hipEventElapsedTime(ms, a, b));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int ftp_options_default(ftp_options* opt) {
  if (!opt) return FTP_E_NULL;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = FTP_FP32_SUMS;
  opt->solver = FTP_SOLVER_PLAIN;
  opt->nfft_R = 2.0;
  opt->nfft_msp = 0;
  opt->solve_waves = 0;
  opt->flags = 0;
  return FTP_OK;
}

}  // extern "C"

namespace {
// Table of the Cayley map theta = phi0 + 2 atan x for degree D < 64: with
// u = 1 + i x, v = 1 - i x, the coefficient of x^c in u^j v^(D-j) is i^c N_c(j),
// N_c(j) = sum_a (-1)^(c-a) C(j, a) C(D-j, c-a) (an integer, |N_c(j)| <= C(D, c)),
// so f_c = Re(i^c sum_j rho_{j-K} N_c(j)) is rho.x (c even) or rho.y (c odd)
// against N_c, with the sign of i^c's real or imaginary part.  Stored as
// T[j (D + 1) + c] = s_c N_c(j), s_c = +1 for c = 0, 3 mod 4 and -1 for 1, 2.
// Exact integers up to D = 52; the entries of larger D round to doubles.
// Only rows j = 0..K (D = 2K) are kept: N_c(D - j) = (-1)^c N_c(j) (a -> c - a
// in the sum), and rho_{D-j} = conj(rho_j) since R is real, so the terms j and
// D - j of f_c are equal and f_c = sum_{j<K} 2 rho'_j T[j][c] + rho'_K T[K][c].
std::vector<double> cayley_table(int D) {
  std::vector<std::vector<int64_t>> C(D + 1, std::vector<int64_t>(D + 1, 0));
  for (int n = 0; n <= D; ++n) {
    C[n][0] = 1;
    for (int k = 1; k <= n; ++k) C[n][k] = C[n - 1][k - 1] + (k <= n - 1 ? C[n - 1][k] : 0);
  }
  const int K = D / 2;
  std::vector<double> T((size_t)(K + 1) * (D + 1));
  for (int j = 0; j <= K; ++j)
    for (int c = 0; c <= D; ++c) {
      int64_t acc = 0;
      const int a0 = c - (D - j) > 0 ? c - (D - j) : 0, a1 = j < c ? j : c;
      for (int a = a0; a <= a1; ++a) {
        const int64_t t = C[j][a] * C[D - j][c - a];
        acc += ((c - a) & 1) ? -t : t;
      }
      const double sgn = (c % 4 == 0 || c % 4 == 3) ? 1.0 : -1.0;
      T[(size_t)j * (D + 1) + c] = sgn * (double)acc;
    }
  return T;
}

// Plan for one template (n_band = 0) or for n_band band templates (c, s of
// n_band x H, band-major; shared-phase calls).
int plan_create_impl(ftp_plan** out, int n_band, int H, const double* c, const double* s, const ftp_options* opt) {
  if (!out) return FTP_E_NULL;
  *out = nullptr;
  int rc;
  const int nt = n_band > 0 ? n_band : 1;
  if (!c || !s) return FTP_E_NULL;
  bool any = false;
  for (int b = 0; b < nt; ++b) {
    rc = validate_template(H, c + b * H, s + b * H);
    if (rc == FTP_OK) any = true;
    else if (rc != FTP_E_H || n_band == 0) return rc;
    for (int n = 0; n < H; ++n)
      if (!std::isfinite(c[b * H + n]) || !std::isfinite(s[b * H + n])) return FTP_E_H;
  }
  if (!any) return FTP_E_H;
  if (H < 1 || H > FTP_MAX_H) return FTP_E_H;
  ftp_options o;
  if (opt) o = *opt; else ftp_options_default(&o);
  if (o.precision != FTP_FP32_SUMS && o.precision != FTP_FP64) return FTP_E_OPTION;
  if (o.solver < FTP_SOLVER_PLAIN || o.solver > FTP_SOLVER_ABERTH) return FTP_E_OPTION;
  if (o.solver == FTP_SOLVER_ABERTH && 6 * H - 2 > 64) return FTP_E_OPTION;   // one root per lane
  if (o.nfft_R != 0.0 && !(o.nfft_R >= 1.5 && o.nfft_R <= 16.0)) return FTP_E_OPTION;
  if (o.nfft_msp < 0 || o.nfft_msp > 24) return FTP_E_OPTION;
  if (o.solve_waves < 0) return FTP_E_OPTION;
  ftp_plan* P = new ftp_plan();
  P->H = H;
  P->n_band = n_band;
  P->opt = o;
  P->c.assign(c, c + nt * H);
  P->s.assign(s, s + nt * H);
  hipError_t e = hipGetDevice(&P->device);
  if (e == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) {
      P->n_cu = prop.multiProcessorCount;
      P->arch = prop.gcnArchName;
      const size_t colon = P->arch.find(':');
      if (colon != std::string::npos) P->arch.resize(colon);
    }
  }
  if (e != hipSuccess) { g_last_error = hipGetErrorString(e); delete P; return FTP_E_HIP; }
  {
    // chunk sizes from the device's free memory at creation: NFFT grids of a
    // ragged batch up to a quarter of it (8..48 GiB; 288 GB of HBM holds a
    // 4096-lightcurve batch's grids in one chunk), per-pair records up to
    // 4 GiB per solve round (2^21 .. 2^23 pairs)
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) {
      P->grid_budget = std::min<size_t>(std::max<size_t>(free_b / 4, (size_t)8 << 30), (size_t)48 << 30);
    }
    const size_t rec_bytes = sizeof(double) * (size_t)RecLayout(H).stride;
    int64_t pc = (int64_t)1 << 21;
    while (pc < ((int64_t)1 << 23) && (size_t)(2 * pc) * rec_bytes <= ((size_t)4 << 30)) pc *= 2;
    P->pair_chunk = pc;
  }
  std::vector<double2> al(nt * H);
  for (int n = 0; n < nt * H; ++n) al[n] = make_double2(0.5 * c[n], 0.5 * s[n]);
  std::vector<float2> tw32(kTwiddleN);
  std::vector<double2> tw64(kTwiddleN);
  for (int k = 0; k < kTwiddleN; ++k) {
    const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)kTwiddleN;
    tw64[k] = make_double2((double)cosl(ang), (double)sinl(ang));
    tw32[k] = make_float2((float)tw64[k].x, (float)tw64[k].y);
  }
  if ((rc = P->alpha.ensure(sizeof(double2) * nt * H)) || (rc = P->twiddle32.ensure(sizeof(float2) * kTwiddleN)) ||
      (rc = P->twiddle64.ensure(sizeof(double2) * kTwiddleN)) || (rc = P->counters.ensure(sizeof(SolveCounters) * kCounterSlots))) {
    delete P;
    return rc;
  }
  if (hipMemcpy(P->alpha.p, al.data(), sizeof(double2) * nt * H, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->twiddle32.p, tw32.data(), sizeof(float2) * kTwiddleN, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->twiddle64.p, tw64.data(), sizeof(double2) * kTwiddleN, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(P->counters.p, 0, sizeof(SolveCounters) * kCounterSlots) != hipSuccess ||
      hipEventCreateWithFlags(&P->upload_done, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&P->fork_ev) != hipSuccess || hipEventCreate(&P->join_ev) != hipSuccess) {
    g_last_error = "plan setup copy failed";
    delete P;
    return FTP_E_HIP;
  }
  const int D = 6 * H - 2;
  if (D < 64) {
    std::vector<double> ct = cayley_table(D);
    if ((rc = P->ctab.ensure(sizeof(double) * ct.size()))) {
      delete P;
      return rc;
    }
    if (hipMemcpy(P->ctab.p, ct.data(), sizeof(double) * ct.size(), hipMemcpyHostToDevice) != hipSuccess) {
      g_last_error = "plan setup copy failed";
      delete P;
      return FTP_E_HIP;
    }
  }
  *out = P;
  return FTP_OK;
}
}  // namespace

extern "C" {

int ftp_plan_create(ftp_plan** out, int H, const double* c, const double* s, const ftp_options* opt) {
  if (!out) return FTP_E_NULL;
  *out = nullptr;
  int rc = validate_template(H, c, s);
  if (rc) return rc;
  return plan_create_impl(out, 0, H, c, s, opt);
}

int ftp_plan_create_bands(ftp_plan** out, int n_band, int H, const double* c, const double* s,
                          const ftp_options* opt) {
  if (!out) return FTP_E_NULL;
  *out = nullptr;
  if (n_band < 1 || n_band > kMaxBands) return FTP_E_OPTION;
  return plan_create_impl(out, n_band, H, c, s, opt);
}

int ftp_plan_destroy(ftp_plan* P) {
  if (!P) return FTP_E_NULL;
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&P->alpha, &P->twiddle32, &P->twiddle64, &P->ctab, &P->d_stage,
                    &P->pw, &P->py, &P->tile_count, &P->tile_off, &P->cursor,
                    &P->block_sums, &P->total, &P->bucket, &P->grids,
                    &P->counters, &P->stats_out, &P->rec, &P->stat_part, &P->stat_ticket, &P->xfeat, &P->seeds, &P->fb_list,
                    &P->fb2_list, &P->rt_list, &P->work_ctr, &P->tune_out, &P->mb_out, &P->mb_chi2};
  P->net.release();
  for (DevBuf* b : bufs) b->release();
  if (P->upload_done) (void)hipEventDestroy(P->upload_done);
  if (P->fork_ev) (void)hipEventDestroy(P->fork_ev);
  if (P->join_ev) (void)hipEventDestroy(P->join_ev);
  if (P->side) (void)hipStreamDestroy(P->side);
  if (P->h_stage) (void)hipHostFree(P->h_stage);
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : P->evr) (void)hipEventDestroy(e);
  for (hipEvent_t e : P->evl) (void)hipEventDestroy(e);
  for (hipEvent_t e : P->evn) (void)hipEventDestroy(e);
  delete P;
  return FTP_OK;
}

int ftp_periodogram(ftp_plan* P, const double* t, const double* y, const double* sigma, int64_t n_obs,
                    double df, int64_t n_f, double* power, double* phase, double* amp, double* offset,
                    uint8_t* status, void* stream) {
  if (!P || !t || !y || !sigma || !power || !phase || !amp || !offset) return FTP_E_NULL;
  int rc = validate_scalars(df, n_f, n_obs);
  if (rc) return rc;
  const int64_t obs_off[2] = {0, n_obs};
  const int64_t freq_off[2] = {0, n_f};
  return run_batch(P, 1, obs_off, t, y, sigma, &df, freq_off, power, phase, amp, offset, status, nullptr,
                   (hipStream_t)stream);
}

int ftp_periodogram_batch(ftp_plan* P, int64_t n_lc, const int64_t* obs_off, const double* t, const double* y,
                          const double* sigma, const double* df, const int64_t* freq_off, double* power,
                          double* phase, double* amp, double* offset, uint8_t* status, void* stream) {
  if (!P || !obs_off || !t || !y || !sigma || !df || !freq_off || !power || !phase || !amp || !offset)
    return FTP_E_NULL;
  if (n_lc < 1) return FTP_E_OFFSETS;
  if (obs_off[0] != 0 || freq_off[0] != 0) return FTP_E_OFFSETS;
  for (int64_t b = 0; b < n_lc; ++b) {
    if (obs_off[b + 1] < obs_off[b] || freq_off[b + 1] < freq_off[b]) return FTP_E_OFFSETS;
    int rc = validate_scalars(df[b], freq_off[b + 1] - freq_off[b], obs_off[b + 1] - obs_off[b]);
    if (rc) return rc;
  }
  if (obs_off[n_lc] > ((int64_t)1 << 30)) return FTP_E_SIZE;
  return run_batch(P, n_lc, obs_off, t, y, sigma, df, freq_off, power, phase, amp, offset, status, nullptr,
                   (hipStream_t)stream);
}

int ftp_periodogram_multiband(ftp_plan* P, int64_t n_band, const int64_t* obs_off, const double* t, const double* y,
                              const double* sigma, double df, int64_t n_f, double* power, double* band_power,
                              double* chi2_0, void* stream) {
  if (!P || !obs_off || !t || !y || !sigma || !power) return FTP_E_NULL;
  if (n_band < 1) return FTP_E_OFFSETS;
  if (obs_off[0] != 0) return FTP_E_OFFSETS;
  for (int64_t b = 0; b < n_band; ++b) {
    if (obs_off[b + 1] < obs_off[b]) return FTP_E_OFFSETS;
    int rc = validate_scalars(df, n_f, obs_off[b + 1] - obs_off[b]);
    if (rc) return rc;
  }
  if (obs_off[n_band] > ((int64_t)1 << 30)) return FTP_E_SIZE;
  if (n_f > (((int64_t)1 << 40) / n_band)) return FTP_E_SIZE;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = n_band * n_f;
  int rc;
  // band outputs: power (caller's band_power or scratch), phase, amp, offset, status
  if ((rc = P->mb_out.ensure((size_t)np * (4 * sizeof(double) + 1)))) return rc;
  if ((rc = P->mb_chi2.ensure(sizeof(double) * n_band))) return rc;
  double* scr = P->mb_out.as<double>();
  double* bp = band_power ? band_power : scr;
  double* c2 = chi2_0 ? chi2_0 : P->mb_chi2.as<double>();
  std::vector<int64_t> freq_off(n_band + 1);
  std::vector<double> dfs(n_band, df);
  for (int64_t b = 0; b <= n_band; ++b) freq_off[b] = b * n_f;
  P->lc_chi2_out = c2;
  rc = run_batch(P, n_band, obs_off, t, y, sigma, dfs.data(), freq_off.data(), bp, scr + np, scr + 2 * np,
                 scr + 3 * np, reinterpret_cast<uint8_t*>(scr + 4 * np), nullptr, st);
  P->lc_chi2_out = nullptr;
  if (rc) return rc;
  HIP_TRY(launch_mb_combine(bp, n_band, n_f, c2, power, st));
  return FTP_OK;
}

int ftp_periodogram_shared_phase(ftp_plan* P, const int64_t* obs_off, const double* t, const double* y,
                                 const double* sigma, const double* offsets, double df, int64_t n_f, double* power,
                                 double* phase, double* amp, double* offset, uint8_t* status, void* stream) {
  if (!P || !obs_off || !t || !y || !sigma || !power || !phase || !amp || !offset) return FTP_E_NULL;
  const int nb = P->n_band;
  if (nb < 1) return FTP_E_OPTION;
  if (obs_off[0] != 0) return FTP_E_OFFSETS;
  for (int b = 0; b < nb; ++b) {
    if (obs_off[b + 1] < obs_off[b]) return FTP_E_OFFSETS;
    if (obs_off[b + 1] == obs_off[b]) return FTP_E_NOBS;
    if (offsets && !std::isfinite(offsets[b])) return FTP_E_OPTION;
  }
  int rc = validate_scalars(df, n_f, obs_off[nb]);
  if (rc) return rc;
  if (obs_off[nb] > ((int64_t)1 << 30)) return FTP_E_SIZE;
  if (P->opt.solver == FTP_SOLVER_LEARNED && !P->mlp_loaded) return FTP_E_NO_MODEL;
  if (n_f > (((int64_t)1 << 40) / nb)) return FTP_E_SIZE;
  if ((rc = wait_uploads(P))) return rc;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int64_t> freq_off(nb + 1);
  std::vector<double> dfs(nb, df);
  for (int b = 0; b <= nb; ++b) freq_off[b] = (int64_t)b * n_f;
  int64_t n_grid = 0, n_tiles = 0;
  if ((rc = plan_chunk(P, 0, nb, obs_off, dfs.data(), freq_off.data(), &n_grid, &n_tiles))) return rc;
  for (int b = 0; b < nb; ++b) P->h_lc[b].yoff = offsets ? offsets[b] : 0.0;
  if ((rc = upload_tables(P, nb, st, true))) return rc;
  hipEvent_t e0 = next_event(P);
  if (e0) HIP_TRY(hipEventRecord(e0, st));
  if (P->opt.precision == FTP_FP64)
    rc = run_nfft<double>(P, nb, obs_off[nb], n_grid, n_tiles, nb, t, y, sigma, st);
  else
    rc = run_nfft<float>(P, nb, obs_off[nb], n_grid, n_tiles, nb, t, y, sigma, st);
  if (rc) return rc;
  hipEvent_t e1 = next_event(P);
  if (e1) HIP_TRY(hipEventRecord(e1, st));
  SolveArgs a = base_args(P, 1, n_f);
  a.n_band = nb;
  a.power = power;
  a.phase = phase;
  a.amp = amp;
  a.offset = offset;
  a.status = status;
  if ((rc = run_solve(P, a, n_f, st))) return rc;
  hipEvent_t e2 = next_event(P);
  if (e2) HIP_TRY(hipEventRecord(e2, st));
  P->last.n_pairs += (uint64_t)n_f;
  return FTP_OK;
}

int ftp_nfft_sums(ftp_plan* P, const double* t, const double* y, const double* sigma, int64_t n_obs, double df,
                  int64_t n_f, double* sums, double* lc_stats, void* stream) {
  if (!P || !t || !y || !sigma || !sums || !lc_stats) return FTP_E_NULL;
  int rc = validate_scalars(df, n_f, n_obs);
  if (rc) return rc;
  const int64_t obs_off[2] = {0, n_obs};
  const int64_t freq_off[2] = {0, n_f};
  rc = run_batch(P, 1, obs_off, t, y, sigma, &df, freq_off, nullptr, nullptr, nullptr, nullptr, nullptr, sums,
                 (hipStream_t)stream);
  if (rc) return rc;
  // lc_stats: tref, ybar, yy, status bits
  HIP_TRY(launch_export_stats(P->d_lc, lc_stats, (hipStream_t)stream));
  return FTP_OK;
}

int ftp_solve_sums(ftp_plan* P, const double* sums, const double* lc_stats, double df, int64_t n_f, double* power,
                   double* phase, double* amp, double* offset, uint8_t* status, void* stream) {
  if (!P || !sums || !lc_stats || !power || !phase || !amp || !offset) return FTP_E_NULL;
  if (!(std::isfinite(df) && df > 0.0)) return FTP_E_DF;
  if (n_f < 1) return FTP_E_NF;
  if (!(lc_stats[2] > 0.0) || !std::isfinite(lc_stats[0]) || !std::isfinite(lc_stats[1])) return FTP_E_OPTION;
  int rc;
  if (P->opt.solver == FTP_SOLVER_LEARNED && !P->mlp_loaded) return FTP_E_NO_MODEL;
  if (P->n_band) return FTP_E_OPTION;
  if ((rc = wait_uploads(P))) return rc;
  hipStream_t st = (hipStream_t)stream;
  P->h_lc.assign(1, LcInfo{});
  LcInfo& L = P->h_lc[0];
  L.n_f = n_f;
  L.df = df;
  L.tref = lc_stats[0];
  L.ybar = lc_stats[1];
  L.yy = lc_stats[2];
  L.inv_sqrt_yy = 1.0 / std::sqrt(lc_stats[2]);
  P->h_obs_off.assign(2, 0);
  P->h_freq_off = {0, n_f};
  P->h_lcb.clear();
  P->h_gtb.assign(3, 0);
  if ((rc = upload_tables(P, 1, st, false))) return rc;
  SolveArgs a = base_args(P, 1, n_f);
  a.sums_in = sums;
  a.mm_tau = 1e-14;
  a.power = power;
  a.phase = phase;
  a.amp = amp;
  a.offset = offset;
  a.status = status;
  if ((rc = run_solve(P, a, n_f, st))) return rc;
  P->last.n_pairs += (uint64_t)n_f;
  return FTP_OK;
}

}  // extern "C"

// ------------------------------------------------- entry point without allocation
// ftp_solve_sums_noalloc keeps all of its scratch (the lightcurve table, the
// work counters, the per-pair records and work lists) in this array: one copy
// per GPU, held by the loaded code object until the process ends.  In host
// code the name is a host-side stand-in, not a device address; each GPU's
// address is looked up once (hipGetSymbolAddress with that GPU current) and
// only that address is passed to kernels.
namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr size_t kNoAllocHead = 4096;   // lightcurve table (1 KB), offsets, counters
constexpr int kNoAllocDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocDevices] = {};

// Address of this GPU's scratch (looked up on the first call per device).
int noalloc_scratch(int device, unsigned char** out) {
  if (device < 0 || device >= kNoAllocDevices) return FTP_E_OPTION;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      g_last_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return FTP_E_HIP;
    }
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return FTP_OK;
}

// The one-lightcurve table of a solve from given sums, written on the device
// (no host staging): every field zero except n_f, df, t_ref, ybar, YY.
__global__ void k_noalloc_tables(LcInfo* lc, int64_t* freq_off, int64_t n_f, double df, double tref, double ybar,
                                 double yy) {
  if (threadIdx.x != 0) return;
  LcInfo L{};
  L.n_f = n_f;
  L.df = df;
  L.tref = tref;
  L.ybar = ybar;
  L.yy = yy;
  L.inv_sqrt_yy = 1.0 / sqrt(yy);
  *lc = L;
  freq_off[0] = 0;
  freq_off[1] = n_f;
}

}  // namespace

extern "C" {

int ftp_solve_sums_noalloc(ftp_plan* P, const double* sums, const double* lc_stats, double df, int64_t n_f,
                           double* power, double* phase, double* amp, double* offset, uint8_t* status,
                           void* stream) {
  if (!P || !sums || !lc_stats || !power || !phase || !amp || !offset) return FTP_E_NULL;
  if (!(std::isfinite(df) && df > 0.0)) return FTP_E_DF;
  if (n_f < 1) return FTP_E_NF;
  if (!(lc_stats[2] > 0.0) || !std::isfinite(lc_stats[0]) || !std::isfinite(lc_stats[1]) ||
      !std::isfinite(lc_stats[2]))
    return FTP_E_OPTION;
  if (P->n_band || P->opt.solver == FTP_SOLVER_LEARNED) return FTP_E_OPTION;
  const RecLayout RL(P->H);
  const size_t per_pair = sizeof(double) * (size_t)RL.stride + 3 * sizeof(int64_t);
  const int64_t cap = (int64_t)((kNoAllocBytes - kNoAllocHead) / per_pair);
  if (cap < 1) return FTP_E_SIZE;
  unsigned char* base = nullptr;
  int rc;
  if ((rc = noalloc_scratch(P->device, &base))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t chunk = std::min<int64_t>(n_f, cap);
  LcInfo* d_lc = reinterpret_cast<LcInfo*>(base);
  int64_t* d_foff = reinterpret_cast<int64_t*>(base + 1024);
  SolveBufs B{};
  B.ctr = reinterpret_cast<unsigned*>(base + 2048);
  B.rec = reinterpret_cast<double*>(base + kNoAllocHead);
  B.fb_list = reinterpret_cast<int64_t*>(base + kNoAllocHead + sizeof(double) * (size_t)RL.stride * chunk);
  B.fb2_list = B.fb_list + chunk;
  B.rt_list = B.fb2_list + chunk;
  B.chunk = chunk;
  B.counters = nullptr;
  B.timing = false;
  hipLaunchKernelGGL(k_noalloc_tables, dim3(1), dim3(64), 0, st, d_lc, d_foff, n_f, df, lc_stats[0], lc_stats[1],
                     lc_stats[2]);
  HIP_TRY(hipGetLastError());
  SolveArgs a = base_args(P, 1, n_f);
  a.lcs = d_lc;
  a.freq_off = d_foff;
  a.grids = nullptr;
  a.sums_in = sums;
  a.mm_tau = 1e-14;
  a.power = power;
  a.phase = phase;
  a.amp = amp;
  a.offset = offset;
  a.status = status;
  if ((rc = run_solve_with(P, a, n_f, B, st))) return rc;
  P->last.n_pairs += (uint64_t)n_f;
  return FTP_OK;
}

int ftp_root_counts(ftp_plan* P, const double* sums, const double* lc_stats, double df, int64_t n_f,
                    int32_t* sturm_count, int32_t* companion_real, void* stream) {
  if (!P || !sums || !lc_stats || !sturm_count || !companion_real) return FTP_E_NULL;
  if (!(std::isfinite(df) && df > 0.0)) return FTP_E_DF;
  if (n_f < 1) return FTP_E_NF;
  if (!(lc_stats[2] > 0.0) || !std::isfinite(lc_stats[0]) || !std::isfinite(lc_stats[1])) return FTP_E_OPTION;
  if (P->n_band) return FTP_E_OPTION;
  int rc;
  if ((rc = wait_uploads(P))) return rc;
  hipStream_t st = (hipStream_t)stream;
  P->h_lc.assign(1, LcInfo{});
  LcInfo& L = P->h_lc[0];
  L.n_f = n_f;
  L.df = df;
  L.tref = lc_stats[0];
  L.ybar = lc_stats[1];
  L.yy = lc_stats[2];
  L.inv_sqrt_yy = 1.0 / std::sqrt(lc_stats[2]);
  P->h_obs_off.assign(2, 0);
  P->h_freq_off = {0, n_f};
  P->h_lcb.clear();
  P->h_gtb.assign(3, 0);
  if ((rc = upload_tables(P, 1, st, false))) return rc;
  SolveArgs a = base_args(P, 1, n_f);
  a.sums_in = sums;
  a.mm_tau = 1e-14;
  const RecLayout RL(P->H);
  const int64_t chunk = std::min<int64_t>(n_f, P->pair_chunk);
  if ((rc = P->rec.ensure(sizeof(double) * (size_t)chunk * RL.stride))) return rc;
  if ((rc = P->work_ctr.ensure(8 * sizeof(unsigned)))) return rc;
  double* rec = P->rec.as<double>();
  unsigned* ctr = P->work_ctr.as<unsigned>();
  for (int64_t p0 = 0; p0 < n_f; p0 += chunk) {
    const int64_t np = std::min<int64_t>(chunk, n_f - p0);
    SolveArgs aa = a;
    aa.clear8 = ctr;
    HIP_TRY(launch_assemble(P->opt.precision, aa, rec, p0, np, (int)grid_waves(P, P->tune.assemble_wpc, np), st));
    HIP_TRY(launch_qr(P->H, rec, RL.stride, np, nullptr, nullptr, P->counters.as<SolveCounters>(), ctr + 4,
                      (int)grid_waves(P, P->tune.qr_wpc, np), st));
    HIP_TRY(launch_root_counts(rec, P->H, np, sturm_count + p0, companion_real + p0,
                               (int)grid_waves(P, P->tune.newton_wpc, np), st));
  }
  return FTP_OK;
}

int ftp_plan_load_mlp(ftp_plan* P, const float* weights, int64_t n_floats, int width) {
  if (!P || !weights) return FTP_E_NULL;
  if (width < 16 || width > 1024 || width % 16) return FTP_E_SIZE;
  MlpNet& N = P->net;
  N.din = 2 * (6 * P->H - 1);
  N.width = width;
  N.dout = 4 * P->H;
  N.layout();
  if (n_floats != N.n_params) return FTP_E_SIZE;
  int rc = mlp_set_weights(&N, weights);
  if (rc) return rc;
  if ((rc = mlp_build_inference(&N, weights))) return rc;
  P->mlp_loaded = true;
  return FTP_OK;
}


struct ftp_mlp {
  MlpNet net;
};

int ftp_mlp_create(ftp_mlp** out, int d_in, int width, int d_out, const float* weights, uint64_t seed) {
  if (!out) return FTP_E_NULL;
  *out = nullptr;
  if (d_in < 1 || d_in > 4096 || width < 16 || width > 1024 || width % 16 || d_out < 2 || d_out > 48 ||
      d_out % 2)
    return FTP_E_SIZE;
  ftp_mlp* M = new ftp_mlp();
  MlpNet& N = M->net;
  N.din = d_in;
  N.width = width;
  N.dout = d_out;
  N.layout();
  std::vector<float> w(N.n_params, 0.f);
  if (weights) {
    std::memcpy(w.data(), weights, sizeof(float) * N.n_params);
  } else {
    // He-uniform weights, zero biases (splitmix64 stream)
    uint64_t x = seed;
    auto next = [&x]() {
      x += 0x9e3779b97f4a7c15ull;
      uint64_t z = x;
      z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
      z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
      return z ^ (z >> 31);
    };
    for (int l = 0; l < 4; ++l) {
      const double lim = std::sqrt(6.0 / N.nin[l]);
      for (int64_t i = 0; i < (int64_t)N.nin[l] * N.nout[l]; ++i) {
        const double u = (double)(next() >> 11) * (1.0 / 9007199254740992.0);
        w[N.oW[l] + i] = (float)((2.0 * u - 1.0) * lim);
      }
    }
  }
  int rc = mlp_set_weights(&N, w.data());
  if (!rc) rc = N.am.ensure(sizeof(float) * N.n_params);
  if (!rc) rc = N.av.ensure(sizeof(float) * N.n_params);
  if (!rc) rc = N.grad.ensure(sizeof(float) * N.n_params);
  if (!rc && (hipMemset(N.am.p, 0, sizeof(float) * N.n_params) != hipSuccess ||
              hipMemset(N.av.p, 0, sizeof(float) * N.n_params) != hipSuccess))
    rc = FTP_E_HIP;
  if (rc) {
    N.release();
    delete M;
    return rc;
  }
  *out = M;
  return FTP_OK;
}

int ftp_mlp_destroy(ftp_mlp* M) {
  if (!M) return FTP_E_NULL;
  (void)hipDeviceSynchronize();
  M->net.release();
  delete M;
  return FTP_OK;
}

int ftp_mlp_num_params(const ftp_mlp* M, int64_t* n) {
  if (!M || !n) return FTP_E_NULL;
  *n = M->net.n_params;
  return FTP_OK;
}

int ftp_mlp_get_weights(ftp_mlp* M, float* host, int64_t n) {
  if (!M || !host) return FTP_E_NULL;
  if (n != M->net.n_params) return FTP_E_SIZE;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(host, M->net.w32.p, sizeof(float) * n, hipMemcpyDeviceToHost));
  return FTP_OK;
}

int ftp_mlp_forward(ftp_mlp* M, const uint16_t* X, int64_t B, float* out, void* stream) {
  if (!M || !X || !out) return FTP_E_NULL;
  if (B < 1) return FTP_E_SIZE;
  int rc = M->net.ensure_batch(B);
  if (rc) return rc;
  return mlp_forward(&M->net, X, B, out, (hipStream_t)stream);
}

int ftp_mlp_loss_grad(ftp_mlp* M, const uint16_t* X, int64_t B, const float* roots, const int* nroots, int R,
                      float lam, float* loss, float* grads, void* stream) {
  if (!M || !X || !roots || !nroots) return FTP_E_NULL;
  if (B < 1 || R < 1) return FTP_E_SIZE;
  hipStream_t st = (hipStream_t)stream;
  int rc = mlp_loss_grad(&M->net, X, B, roots, nroots, R, lam, st);
  if (rc) return rc;
  if (loss) HIP_TRY(hipMemcpyAsync(loss, M->net.loss.p, sizeof(float) * B, hipMemcpyDeviceToDevice, st));
  if (grads)
    HIP_TRY(hipMemcpyAsync(grads, M->net.grad.p, sizeof(float) * M->net.n_params, hipMemcpyDeviceToDevice, st));
  return FTP_OK;
}

int ftp_mlp_train_step(ftp_mlp* M, const uint16_t* X, int64_t B, const float* roots, const int* nroots, int R,
                       float lam, float lr, float* loss, void* stream) {
  if (!M || !X || !roots || !nroots) return FTP_E_NULL;
  if (B < 1 || R < 1 || !(lr > 0.f)) return FTP_E_SIZE;
  hipStream_t st = (hipStream_t)stream;
  MlpNet& N = M->net;
  int rc = mlp_loss_grad(&N, X, B, roots, nroots, R, lam, st);
  if (rc) return rc;
  N.step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)N.step), c2 = 1.f - std::pow(b2, (float)N.step);
  HIP_TRY(launch_adam(N.w32.as<float>(), N.wbf.as<uint16_t>(), N.grad.as<float>(), N.am.as<float>(),
                      N.av.as<float>(), N.n_params, lr, b1, b2, 1e-8f, c1, c2, st));
  if (loss) HIP_TRY(hipMemcpyAsync(loss, N.loss.p, sizeof(float) * B, hipMemcpyDeviceToDevice, st));
  return FTP_OK;
}

int ftp_learned_dataset(ftp_plan* P, const double* t, const double* y, const double* sigma, int64_t n_obs,
                        double df, int64_t n_f, uint16_t* X, float* roots, int* nroots, int R, void* stream) {
  if (!P || !t || !y || !sigma || !X || !roots || !nroots) return FTP_E_NULL;
  int rc = validate_scalars(df, n_f, n_obs);
  if (rc) return rc;
  if (R < 1 || R > 64) return FTP_E_SIZE;
  if (P->n_band) return FTP_E_OPTION;
  const int64_t obs_off[2] = {0, n_obs};
  const int64_t freq_off[2] = {0, n_f};
  P->ds_X = X;
  P->ds_roots = roots;
  P->ds_nroots = nroots;
  P->ds_R = R;
  rc = run_batch(P, 1, obs_off, t, y, sigma, &df, freq_off, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                 (hipStream_t)stream);
  P->ds_X = nullptr;
  P->ds_roots = nullptr;
  P->ds_nroots = nullptr;
  return rc;
}

int ftp_plan_get_tuning(const ftp_plan* P, ftp_tuning* out) {
  if (!P || !out) return FTP_E_NULL;
  *out = P->tune;
  return FTP_OK;
}

int ftp_plan_set_tuning(ftp_plan* P, const ftp_tuning* t) {
  if (!P || !t) return FTP_E_NULL;
  if (!tuning_valid(*t)) return FTP_E_OPTION;
  P->tune = *t;
  return FTP_OK;
}

int ftp_plan_tune_key(const ftp_plan* P, int64_t n_f, char* buf, int len) {
  if (!P || !buf) return FTP_E_NULL;
  if (n_f < 1) return FTP_E_NF;
  // frequency-count bucket: even powers of two (2^(2b) <= n_f < 2^(2b+2)),
  // 2^10 .. 2^24 and beyond in one bucket
  int lg = 0;
  while (lg < 62 && ((int64_t)1 << (lg + 1)) <= n_f) ++lg;
  const int bucket = std::min(std::max(lg & ~1, 10), 24);
  const int n = std::snprintf(buf, len > 0 ? (size_t)len : 0, "%s/%dcu/H%d/p%d/s%d/nf%d", P->arch.c_str(),
                              P->n_cu, P->H, P->opt.precision, P->opt.solver, bucket);
  if (n < 0 || n >= len) return FTP_E_SIZE;
  return FTP_OK;
}

int ftp_tune_cache_lookup(const char* path, const char* key, ftp_tuning* out) {
  if (!path || !out) return FTP_E_NULL;
  if (!key_valid(key)) return FTP_E_OPTION;
  std::ifstream in(path);
  if (!in) return 0;
  std::string line;
  int found = 0;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string k;
    ftp_tuning t{};
    if (!(ls >> k) || k != key) continue;
    if (!(ls >> t.assemble_wpc >> t.newton_wpc >> t.aberth_wpc >> t.qr_wpc >> t.score_wpc >> t.mlp_fused)) continue;
    if (!(ls >> t.newton_occ)) t.newton_occ = 4;
    if (!tuning_valid(t)) continue;
    *out = t;
    found = 1;   // the last well-formed entry wins
  }
  return found;
}

int ftp_tune_cache_store(const char* path, const char* key, const ftp_tuning* t) {
  if (!path || !t) return FTP_E_NULL;
  if (!key_valid(key) || !tuning_valid(*t)) return FTP_E_OPTION;
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line;
    while (in && std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      if ((ls >> k) && k == key) continue;
      if (!line.empty()) keep.push_back(line);
    }
  }
  char entry[512];
  std::snprintf(entry, sizeof(entry), "%s %d %d %d %d %d %d %d", key, t->assemble_wpc, t->newton_wpc, t->aberth_wpc,
                t->qr_wpc, t->score_wpc, t->mlp_fused, t->newton_occ);
  keep.push_back(entry);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return FTP_E_IO;
    for (const std::string& l : keep) out << l << "\n";
    out.flush();
    if (!out) return FTP_E_IO;
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return FTP_E_IO;
  }
  return FTP_OK;
}

int ftp_autotune(ftp_plan* P, const double* t, const double* y, const double* sigma, int64_t n_obs, double df,
                 int64_t n_f, const char* cache_path, unsigned flags, ftp_tuning* out, void* stream) {
  if (!P || !t || !y || !sigma) return FTP_E_NULL;
  int rc = validate_scalars(df, n_f, n_obs);
  if (rc) return rc;
  if (P->opt.solver == FTP_SOLVER_LEARNED && !P->mlp_loaded) return FTP_E_NO_MODEL;
  if (P->n_band) return FTP_E_OPTION;
  char key[256];
  if ((rc = ftp_plan_tune_key(P, n_f, key, (int)sizeof(key)))) return rc;
  if (cache_path && !(flags & FTP_TUNE_FORCE)) {
    ftp_tuning c{};
    rc = ftp_tune_cache_lookup(cache_path, key, &c);
    if (rc < 0) return rc;
    if (rc == 1) {
      P->tune = c;
      if (out) *out = c;
      return 1;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  if ((rc = P->tune_out.ensure((size_t)n_f * (4 * sizeof(double) + 1)))) return rc;
  const ftp_tuning saved = P->tune;
  const unsigned saved_flags = P->opt.flags;
  P->opt.flags &= ~FTP_FLAG_TIME_STAGES;
  ftp_tuning cur = P->tune;
  float ms = 0.f;
  // the knobs that matter for the solver; the QR knob also for the others
  // (it then only serves the companion fallback, but is cheap to sweep)
  int* knobs[7];
  int nk = 0;
  if (P->opt.solver == FTP_SOLVER_PLAIN) {
    knobs[nk++] = &cur.qr_wpc;
  } else {
    if (P->opt.solver != FTP_SOLVER_ABERTH) knobs[nk++] = &cur.newton_wpc;
    knobs[nk++] = &cur.aberth_wpc;
  }
  knobs[nk++] = &cur.assemble_wpc;
  knobs[nk++] = &cur.score_wpc;
  const bool tune_mlp = P->opt.solver == FTP_SOLVER_LEARNED && mlp_fused_ok(P->net.nin, P->net.nout);
  if (tune_mlp) knobs[nk++] = &cur.mlp_fused;
  const bool tune_occ = (P->opt.solver == FTP_SOLVER_LEARNED || P->opt.solver == FTP_SOLVER_UNIFORM) &&
                        newton_four_per_wave(P->H);
  if (tune_occ) knobs[nk++] = &cur.newton_occ;
  // (grids well beyond the resident waves pay for the grid-strided kernels:
  // the dispatcher then balances the uneven per-pair work)
  const int cand[] = {4, 8, 12, 16, 24, 32, 48, 64, 128, 256};
  const int ncand = (int)(sizeof(cand) / sizeof(cand[0]));
  const int cand01[] = {0, 1};
  const int cand_occ[] = {4, 5, 6};
  auto measure = [&](float* best) -> int {
    P->tune = cur;
    float m0 = 0.f, m1 = 0.f;
    int r = time_call(P, t, y, sigma, n_obs, df, n_f, st, &m0);
    if (r) return r;
    r = time_call(P, t, y, sigma, n_obs, df, n_f, st, &m1);
    if (r) return r;
    *best = std::min(m0, m1);
    return FTP_OK;
  };
  rc = time_call(P, t, y, sigma, n_obs, df, n_f, st, &ms);   // warm-up
  for (int k = 0; rc == FTP_OK && k < nk; ++k) {
    int best_v = *knobs[k];
    float best_ms = 0.f;
    if ((rc = measure(&best_ms))) break;
    const bool is_mlp = knobs[k] == &cur.mlp_fused, is_occ = knobs[k] == &cur.newton_occ;
    const int* cv = is_mlp ? cand01 : (is_occ ? cand_occ : cand);
    const int ncv = is_mlp ? 2 : (is_occ ? 3 : ncand);
    for (int ci = 0; ci < ncv; ++ci) {
      const int v = cv[ci];
      if (v == best_v) continue;
      const int keep = *knobs[k];
      *knobs[k] = v;
      float m = 0.f;
      if ((rc = measure(&m))) break;
      if (m < 0.98f * best_ms) {
        best_ms = m;
        best_v = v;
      }
      *knobs[k] = keep;
    }
    *knobs[k] = best_v;
  }
  P->opt.flags = saved_flags;
  if (rc != FTP_OK) {
    P->tune = saved;
    return rc;
  }
  P->tune = cur;
  if (out) *out = cur;
  if (cache_path) {
    const int wr = ftp_tune_cache_store(cache_path, key, &cur);
    if (wr < 0) return wr;
  }
  return 0;
}

int ftp_last_stats(ftp_plan* P, ftp_stats* out, void* stream) {
  if (!P || !out) return FTP_E_NULL;
  SolveCounters cs[kCounterSlots];
  HIP_TRY(hipMemcpyAsync(cs, P->counters.p, sizeof(cs), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  SolveCounters c{};
  for (const SolveCounters& x : cs) {
    c.fallback += x.fallback;
    c.newton_iters += x.newton_iters;
    c.roots_found += x.roots_found;
    c.qr_sweeps += x.qr_sweeps;
    c.aberth_iters += x.aberth_iters;
    c.fallback_qr += x.fallback_qr;
    c.fallback_aberth += x.fallback_aberth;
  }
  *out = P->last;
  out->ms_nfft = 0.0;
  out->ms_solve = 0.0;
  out->ms_roots = 0.0;
  for (int k = 0; k + 3 <= P->ev_used; k += 3) {
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, P->ev[k], P->ev[k + 1]));
    HIP_TRY(hipEventElapsedTime(&b, P->ev[k + 1], P->ev[k + 2]));
    out->ms_nfft += a;
    out->ms_solve += b;
  }
  out->ms_mlp = out->ms_verify = out->ms_retry = out->ms_aberth = out->ms_fallback = 0.0;
  // per chunk: root events (start, end); learned-stage events (after the
  // network, after Newton + Sturm, after Aberth) when the solver has them
  for (int k = 0; k + 2 <= P->evr_used; k += 2) {
    float a = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, P->evr[k], P->evr[k + 1]));
    out->ms_roots += a;
    // learned / uniform / Aberth: after the network on every pair, after
    // the first Newton round, after the network on its list, after the
    // second round, after the Aberth tier
    const int l = 5 * (k / 2);
    if (l + 5 <= P->evl_used) {
      float m = 0.f, v = 0.f, m2 = 0.f, r = 0.f, b = 0.f, f = 0.f;
      HIP_TRY(hipEventElapsedTime(&m, P->evr[k], P->evl[l]));
      HIP_TRY(hipEventElapsedTime(&v, P->evl[l], P->evl[l + 1]));
      HIP_TRY(hipEventElapsedTime(&m2, P->evl[l + 1], P->evl[l + 2]));
      HIP_TRY(hipEventElapsedTime(&r, P->evl[l + 2], P->evl[l + 3]));
      HIP_TRY(hipEventElapsedTime(&b, P->evl[l + 3], P->evl[l + 4]));
      HIP_TRY(hipEventElapsedTime(&f, P->evl[l + 4], P->evr[k + 1]));
      out->ms_mlp += m + m2;
      out->ms_verify += v;
      out->ms_retry += r;
      out->ms_aberth += b;
      out->ms_fallback += f;
    }
  }
  out->ms_spread = out->ms_fft = 0.0;
  for (int k = 0; k + 3 <= P->evn_used; k += 3) {
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, P->evn[k], P->evn[k + 1]));
    HIP_TRY(hipEventElapsedTime(&b, P->evn[k + 1], P->evn[k + 2]));
    out->ms_spread += a;
    out->ms_fft += b;
  }
  out->n_fallback = c.fallback;
  out->n_fallback_qr = c.fallback_qr;
  out->n_fallback_aberth = c.fallback_aberth;
  out->aberth_iters = c.aberth_iters;
  out->qr_sweeps = c.qr_sweeps;
  out->newton_iters = c.newton_iters;
  out->roots_found = c.roots_found;
  // reset the accumulation window
  P->ev_used = 0;
  P->evr_used = 0;
  P->evl_used = 0;
  P->evn_used = 0;
  P->last = ftp_stats{};
  HIP_TRY(hipMemsetAsync(P->counters.p, 0, sizeof(SolveCounters) * kCounterSlots, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return FTP_OK;
}

const char* ftp_status_string(int code) {
  switch (code) {
    case FTP_OK: return "ok";
    case FTP_E_NULL: return "a required pointer is NULL";
    case FTP_E_H: return "invalid template (H out of range, non-finite or all-zero coefficients)";
    case FTP_E_NOBS: return "fewer than 3 observations";
    case FTP_E_DF: return "df must be positive and finite";
    case FTP_E_NF: return "n_f must be at least 1";
    case FTP_E_OFFSETS: return "offsets must start at 0 and be non-decreasing";
    case FTP_E_SIZE: return "size exceeds library limits";
    case FTP_E_HIP: return "HIP runtime error";
    case FTP_E_OPTION: return "invalid option";
    case FTP_E_NO_MODEL: return "learned solver requested but no network is loaded";
    case FTP_E_IO: return "file could not be read or written";
    case FTP_ST_DEGENERATE: return "degenerate frequency (MM ~ 0)";
    case FTP_ST_CONSTANT: return "phase polynomial vanishes (P constant in phase)";
    case FTP_ST_NO_CONVERGE: return "companion QR did not converge";
    case FTP_ST_BAD_LC: return "lightcurve rejected (NaN/Inf, sigma < 0, mixed zero sigma or Var(y) = 0)";
    case FTP_ST_FALLBACK: return "the solver's first method did not settle the frequency (Aberth tier used)";
    case FTP_ST_FALLBACK_QR: return "roots from the companion solve after the Aberth tier";
    default: return "unknown code";
  }
}

const char* ftp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
