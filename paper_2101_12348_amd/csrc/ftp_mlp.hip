// Root-proposal network of the learned solve (a project addition to the
// method): an MLP d_in -> W -> W -> W -> 4H with ReLU, BF16 weights and
// activations, FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16), trained on the device by its own forward and
// backward kernels with Adam on FP32 master weights.
//
// Input features of a frequency: the coefficients p_k, k = 0..D, of the phase
// polynomial (Eq. finalpoly), rotated to a canonical phase (r_1 real and
// positive, where p(e^{i theta}) = -i e^{i K theta} sum_d r_d e^{i d theta}) and
// scaled to max |p_k| = 1, as (Re, Im) pairs: d_in = 2 (D + 1).
// Output: 2H (u, v) pairs; seed k is atan2(v_k, u_k) in the canonical frame.
#include <hip/hip_ext.h>
#include "ftp_solve_common.h"
#include "ftp_args.h"

namespace ftp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;

// float -> bf16 bits by the hardware conversion (round to nearest even, one
// instruction on gfx950; equal to f2bf for finite values), used by the
// inference epilogues of k_dense_bf16 and k_mlp_fused alike
__device__ __forceinline__ uint16_t bf16_rne(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

// ------------------------------------------------------------------ GEMM

// C[m, n] = sum_k A[m, k] B[k, n] with A, B in bf16 at arbitrary strides and
// FP32 accumulation.  Epilogue: + bias[n], optional ReLU, optional ReLU mask
// (C *= (maskB[m, n] > 0) with maskB bf16), FP32 and/or bf16 stores.
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

constexpr int kGT = 64;   // output tile (M and N) per workgroup
constexpr int kGK = 32;   // K step (one MFMA)
constexpr int kGP = 40;   // padded LDS row (bf16 elements)

// 256 threads = 4 waves; wave w owns the 32 x 32 quadrant (w / 2, w % 2) of
// the 64 x 64 tile as 2 x 2 MFMA 16 x 16 x 32 blocks.  Operand fragments (lane
// l): A rows l % 16 with k = 8 (l / 16) .. + 7; B columns l % 16, same k; result
// rows 4 (l / 16) + v, column l % 16 (v = 0..3).
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kGT * kGP];
  __shared__ __align__(16) uint16_t Bs[kGT * kGP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kGT;
  const int n0 = blockIdx.y * kGT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4_t acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int lr = tid >> 2, lk = (tid & 3) * 8;   // loader: row 0..63, k 0/8/16/24
  // 16-byte operand loads when k is contiguous, rows are 16-byte aligned and K
  // is a multiple of the K step
  const bool avec = g.a_k == 1 && (g.a_m & 7) == 0 && (g.K % kGK) == 0 &&
                    ((reinterpret_cast<uintptr_t>(g.A) & 15) == 0);
  const bool bvec = g.b_k == 1 && (g.b_n & 7) == 0 && (g.K % kGK) == 0 &&
                    ((reinterpret_cast<uintptr_t>(g.B) & 15) == 0);
  for (int k0 = 0; k0 < g.K; k0 += kGK) {
    {
      const int64_t m = m0 + lr;
      uint16_t* dst = As + lr * kGP + lk;
      if (avec) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (m < g.M) v = *reinterpret_cast<const uint4*>(g.A + m * g.a_m + k0 + lk);
        *reinterpret_cast<uint4*>(dst) = v;
      } else {
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + lk + q;
          dst[q] = (m < g.M && k < g.K) ? g.A[m * g.a_m + (int64_t)k * g.a_k] : (uint16_t)0;
        }
      }
      const int n = n0 + lr;
      uint16_t* dstb = Bs + lr * kGP + lk;
      if (bvec) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (n < g.N) v = *reinterpret_cast<const uint4*>(g.B + (int64_t)n * g.b_n + k0 + lk);
        *reinterpret_cast<uint4*>(dstb) = v;
      } else {
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + lk + q;
          dstb[q] = (n < g.N && k < g.K) ? g.B[(int64_t)k * g.b_k + (int64_t)n * g.b_n] : (uint16_t)0;
        }
      }
    }
    __syncthreads();
    for (int i = 0; i < 2; ++i) {
      const uint16_t* ap = As + (wm + i * 16 + (lane & 15)) * kGP + 8 * (lane >> 4);
      bf16x8_t af;
      memcpy(&af, ap, 16);
      for (int j = 0; j < 2; ++j) {
        const uint16_t* bp = Bs + (wn + j * 16 + (lane & 15)) * kGP + 8 * (lane >> 4);
        bf16x8_t bfv;
        memcpy(&bfv, bp, 16);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfv, acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i) {
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + j * 16 + (lane & 15);
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm + i * 16 + 4 * (lane >> 4) + v;
        if (m >= g.M || n >= g.N) continue;
        float x = acc[i][j][v];
        if (g.bias) x += g.bias[n];
        if (g.relu) x = fmaxf(x, 0.f);
        if (g.mask) {
          const uint16_t mb = g.mask[m * g.ld_mask + n];
          if ((mb & 0x8000u) || (mb & 0x7fffu) == 0) x = 0.f;
        }
        if (g.Cf) g.Cf[m * g.ld_cf + n] = x;
        if (g.Cb) g.Cb[m * g.ld_cb + n] = f2bf(x);
      }
    }
  }
}

// ------------------------------------------------- inference dense layer

// Y = act(A W^T + b) for inference: A (M x Kp bf16, row stride lda), W (N x Kp
// bf16 row-major), Kp a multiple of 32 (rows zero-padded), 16-byte aligned rows.
// A workgroup of RW x 4 waves owns 64 RW rows and 256 columns (column block
// blockIdx.y); wave (r, c) computes rows 64 r .. + 63 and columns 64 c .. + 63
// of the block as 4 x 4 MFMA 16 x 16 x 32 tiles (64 FP32 accumulators per
// lane).  The K loop stages 32-wide slices of A and W in LDS, double-buffered:
// the global loads of the next slice are issued before the MFMAs of the
// current one; one W slice serves all 64 RW rows.  bf16 outputs leave through
// LDS so that each lane stores 16 contiguous bytes; FP32 outputs (the last
// layer, few columns) are stored directly.
struct DenseArgs {
  const uint16_t* A; int64_t lda;
  const uint16_t* W; int ldw;
  const float* bias;
  int64_t M; int N, Kp;
  int relu;
  uint16_t* Yb; float* Yf; int64_t ldy;
};

constexpr int kDC = 256;   // columns per workgroup
constexpr int kDP = 40;    // padded LDS row (bf16): 80 bytes, rows on distinct banks
#ifndef FTP_DENSE_RW
#define FTP_DENSE_RW 2
#endif
constexpr int kDRW = FTP_DENSE_RW;   // row waves per workgroup

template <int RW>
__global__ __launch_bounds__(256 * RW) void k_dense_bf16(DenseArgs d) {
  constexpr int BM = 64 * RW, NT = 256 * RW;
  __shared__ __align__(16) uint16_t As[2][BM * kDP];
  __shared__ __align__(16) uint16_t Ws[2][kDC * kDP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int c0 = blockIdx.y * kDC;
  const int lr = tid >> 2, lk = (tid & 3) * 8;   // loader: row 0..BM-1, k 0/8/16/24
  constexpr int WQ = kDC / (NT / 4);             // W rows per loader thread
  const bool wave_on = c0 + 64 * wc < d.N;
  f32x4_t acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  uint4 ra, rw[WQ];
  auto load = [&](int k0) {
    const int64_t m = m0 + lr;
    ra = m < d.M ? *reinterpret_cast<const uint4*>(d.A + m * d.lda + k0 + lk) : make_uint4(0u, 0u, 0u, 0u);
    for (int q = 0; q < WQ; ++q) {
      const int n = c0 + lr + BM * q;
      rw[q] = n < d.N ? *reinterpret_cast<const uint4*>(d.W + (int64_t)n * d.ldw + k0 + lk)
                      : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto stage = [&](int b) {
    *reinterpret_cast<uint4*>(&As[b][lr * kDP + lk]) = ra;
    for (int q = 0; q < WQ; ++q) *reinterpret_cast<uint4*>(&Ws[b][(lr + BM * q) * kDP + lk]) = rw[q];
  };
  const int nk = d.Kp / 32;
  load(0);
  stage(0);
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    const int b = ks & 1;
    if (ks + 1 < nk) load(32 * (ks + 1));
    if (wave_on) {
      bf16x8_t af[4], wf[4];
      for (int i = 0; i < 4; ++i)
        memcpy(&af[i], &As[b][(64 * wr + 16 * i + (lane & 15)) * kDP + 8 * (lane >> 4)], 16);
      for (int j = 0; j < 4; ++j)
        memcpy(&wf[j], &Ws[b][(64 * wc + 16 * j + (lane & 15)) * kDP + 8 * (lane >> 4)], 16);
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], wf[j], acc[i][j], 0, 0, 0);
    }
    if (ks + 1 < nk) stage(b ^ 1);
    __syncthreads();
  }
  // lane holds rows 64 wr + 16 i + 4 (lane / 16) + v, column 64 wc + 16 j + lane % 16
  if (d.Yf) {
    if (!wave_on) return;
    for (int j = 0; j < 4; ++j) {
      const int n = c0 + 64 * wc + 16 * j + (lane & 15);
      if (n >= d.N) continue;
      const float bn = d.bias ? d.bias[n] : 0.f;
      for (int i = 0; i < 4; ++i)
        for (int v = 0; v < 4; ++v) {
          const int64_t m = m0 + 64 * wr + 16 * i + 4 * (lane >> 4) + v;
          if (m >= d.M) continue;
          float x = acc[i][j][v] + bn;
          if (d.relu) x = fmaxf(x, 0.f);
          d.Yf[m * d.ldy + n] = x;
        }
    }
    return;
  }
  // bf16: the tile (BM x 256) through LDS, in row slabs of 64 (one per row
  // wave) held in the W buffers (2 x 256 x 40 >= 64 x 264 elements)
  uint16_t* Ct = &Ws[0][0];
  constexpr int kCP = kDC + 8;
  const int ncols = d.N - c0 < kDC ? d.N - c0 : kDC;   // a multiple of 8
  for (int r = 0; r < RW; ++r) {
    if (wr == r && wave_on) {
      for (int j = 0; j < 4; ++j) {
        const int cl = 64 * wc + 16 * j + (lane & 15);
        const float bn = (c0 + cl < d.N && d.bias) ? d.bias[c0 + cl] : 0.f;
        for (int i = 0; i < 4; ++i)
          for (int v = 0; v < 4; ++v) {
            float x = acc[i][j][v] + bn;
            if (d.relu) x = fmaxf(x, 0.f);
            Ct[(16 * i + 4 * (lane >> 4) + v) * kCP + cl] = bf16_rne(x);
          }
      }
    }
    __syncthreads();
    for (int q = tid; q < 64 * (kDC / 8); q += NT) {
      const int rr = q / (kDC / 8), c8 = (q % (kDC / 8)) * 8;
      const int64_t m = m0 + 64 * r + rr;
      if (m >= d.M || c8 >= ncols) continue;
      *reinterpret_cast<uint4*>(d.Yb + m * d.ldy + c0 + c8) = *reinterpret_cast<const uint4*>(&Ct[rr * kCP + c8]);
    }
    __syncthreads();
  }
}

// --------------------------------------------------------- small kernels

// db[n] = sum_m G[m, n] (G fp32, row stride ld)
__global__ __launch_bounds__(256) void k_colsum(const float* G, int64_t M, int N, int64_t ld, float* out) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t m = 0; m < M; ++m) s += G[m * ld + n];
  out[n] = s;
}

// Chamfer loss on the circle between seed vectors e_k = (u_k, v_k) and root
// unit vectors r_j = (cos, sin) (one thread per sample):
//   L_b = (1/n) sum_j min_k |e_k - r_j|^2 + lam (1/K) sum_k min_j |e_k - r_j|^2,
// loss = mean_b L_b; dout = dL/dout (fp32 and bf16).
__global__ __launch_bounds__(256) void k_chamfer(const float* out, int64_t B, int Kseeds, const float* roots,
                                                 const int* nroots, int R, float lam, float* loss_b, float* dout,
                                                 uint16_t* dout_bf) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const float* o = out + b * 2 * Kseeds;
  float g[2 * 24];
  for (int q = 0; q < 2 * Kseeds; ++q) g[q] = 0.f;
  const int n = nroots[b] < R ? nroots[b] : R;
  float L = 0.f;
  const float invB = 1.f / (float)B;
  if (n > 0) {
    for (int jr = 0; jr < n; ++jr) {
      float sn, cs;
      sincosf(roots[b * R + jr], &sn, &cs);
      int kb = 0;
      float db = 3.4e38f;
      for (int k = 0; k < Kseeds; ++k) {
        const float du = o[2 * k] - cs, dv = o[2 * k + 1] - sn;
        const float d2 = du * du + dv * dv;
        if (d2 < db) { db = d2; kb = k; }
      }
      L += db / n;
      g[2 * kb] += 2.f * (o[2 * kb] - cs) / n;
      g[2 * kb + 1] += 2.f * (o[2 * kb + 1] - sn) / n;
    }
    for (int k = 0; k < Kseeds; ++k) {
      float db = 3.4e38f, bu = 0.f, bv = 0.f;
      for (int jr = 0; jr < n; ++jr) {
        float sn, cs;
        sincosf(roots[b * R + jr], &sn, &cs);
        const float du = o[2 * k] - cs, dv = o[2 * k + 1] - sn;
        const float d2 = du * du + dv * dv;
        if (d2 < db) { db = d2; bu = du; bv = dv; }
      }
      L += lam * db / Kseeds;
      g[2 * k] += lam * 2.f * bu / Kseeds;
      g[2 * k + 1] += lam * 2.f * bv / Kseeds;
    }
  }
  loss_b[b] = L;
  for (int q = 0; q < 2 * Kseeds; ++q) {
    const float v = g[q] * invB;
    dout[b * 2 * Kseeds + q] = v;
    dout_bf[b * 2 * Kseeds + q] = f2bf(v);
  }
}

// Adam (Kingma & Ba 2015) on FP32 master weights; writes the bf16 copy.
__global__ __launch_bounds__(256) void k_adam(float* w, uint16_t* wb, const float* g, float* m, float* v,
                                              int64_t n, float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// Network features of pairs [0, np) of a record chunk (one wavefront per
// pair), written to X (row stride ldx >= 2 (D + 1), the rest of the row
// zeroed); the canonical rotation goes to the record for the Newton kernel.
__global__ __launch_bounds__(64) void k_features(double* rec, int H, int64_t np, uint16_t* X, int64_t ldx,
                                                  const int64_t* list, const unsigned* list_count) {
  const RecLayout RL(H);
  const int D = RL.D;
  const int lane = threadIdx.x & 63;
  if (list) np = (int64_t)*list_count;
  for (int64_t i = blockIdx.x; i < np; i += gridDim.x) {
    const int64_t w = list ? list[i] : i;
    double* R = rec + w * (int64_t)RL.stride;
    const int st = (int)R[RL.meta + M_STATUS];
    uint16_t* x = X + i * ldx;
    for (int q = 2 * (D + 1) + lane; q < ldx; q += 64) x[q] = 0;
    if (st == ST_BAD_LC || st == ST_CONSTANT) {
      for (int q = lane; q < 2 * (D + 1); q += 64) x[q] = 0;
      continue;
    }
    const double canon = pair_features(reinterpret_cast<const double2*>(R + RL.r), RL.K, lane, x);
    if (lane == 0) R[RL.meta + M_CANON] = canon;
  }
}

// Two pairs per wavefront (D < 64): the same features, pair 2b on lanes
// 0..31 and 2b + 1 on lanes 32..63, coefficients in two rounds of 32 and the
// scale from a per-half maximum.  Every lane runs the arithmetic (the per-half
// reduction needs the whole wavefront); rejected or constant pairs then write
// zeros instead.
__global__ __launch_bounds__(64) void k_features2(double* rec, int H, int64_t np, uint16_t* X, int64_t ldx,
                                                   const int64_t* list, const unsigned* list_count) {
  const RecLayout RL(H);
  const int D = RL.D, K = RL.K;
  const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  if (list) np = (int64_t)*list_count;
  for (int64_t w0 = 2 * (int64_t)blockIdx.x; w0 < np; w0 += 2 * (int64_t)gridDim.x) {
    const bool has = w0 + half < np;
    const int64_t row = has ? w0 + half : w0;   // row of X
    const int64_t w = list ? list[row] : row;   // pair of the chunk
    double* R = rec + w * (int64_t)RL.stride;
    const int st = (int)R[RL.meta + M_STATUS];
    const bool zero = st == ST_BAD_LC || st == ST_CONSTANT;
    const double2* r = reinterpret_cast<const double2*>(R + RL.r);
    const double2 r1 = r[1];
    const double m1 = sqrt(r1.x * r1.x + r1.y * r1.y);
    const double canon = m1 > 0.0 ? (double)atan2f((float)r1.y, (float)r1.x) : 0.0;
    const double im1 = m1 > 0.0 ? 1.0 / m1 : 0.0;
    const double2 u = m1 > 0.0 ? make_double2(r1.x * im1, -r1.y * im1) : make_double2(1.0, 0.0);
    double2 v[2];
    double a2 = 0.0;   // largest |v|^2 of the half
    for (int s = 0; s < 2; ++s) {
      const int k = hl + 32 * s;
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
      a2 = fmax(a2, v[s].x * v[s].x + v[s].y * v[s].y);
    }
    double lo, hi;
    half_max_d(a2, lo, hi);
    const double amax = sqrt(half ? hi : lo);
    const double sc = amax > 0.0 ? 1.0 / amax : 0.0;
    if (has) {
      // (Re, Im) of coefficient k as one 32-bit store; the padding of the row
      // (ldx and 2 (D + 1) even) likewise
      unsigned* x = reinterpret_cast<unsigned*>(X + row * ldx);
      for (int64_t q = (D + 1) + hl; q < ldx / 2; q += 32) x[q] = 0u;
      for (int s = 0; s < 2; ++s) {
        const int k = hl + 32 * s;
        if (k > D) continue;
        const unsigned re = zero ? 0u : f2bf((float)(v[s].x * sc)), im = zero ? 0u : f2bf((float)(v[s].y * sc));
        x[k] = re | (im << 16);
      }
      if (hl == 0 && !zero) R[RL.meta + M_CANON] = canon;
    }
  }
}

// ------------------------------------------------------- fused inference

// The four layers of the network for kFRows (128 or 32) pairs per workgroup
// (four waves), with the activations kept in LDS between layers: the output of
// a layer is written over its input (after every wave has read it) and is the
// A operand of the next.  Per layer, wave w computes all kFRows rows of the
// column tiles 4w .. 4w + 3 (64 columns) as (kFRows / 16) x 4 MFMA 16 x 16 x 32
// tiles.  The weights (about 300 KB for width 256, resident in L2) are read by
// each wave straight into its B fragments, three K slices ahead, so the K loop
// has no barrier; the LDS holds only the activations (67.5 KB at 128 rows:
// two workgroups per CU).
// Weights: the inference copy with each layer's rows zero-padded to kp[l]
// (multiples of 32, 16-byte aligned) and their number to a multiple of 16.
// Same operands, K order, bias, ReLU and
// bf16 rounding as k_dense_bf16, so the result equals the unfused launches
// bit for bit.  Requirements (checked on the host): width a multiple of 32 up
// to 256, kp[0] up to 256, d_out up to 64.

// kFRows: pairs per workgroup, 128 when the network runs on every pair of a
// round (each workgroup's weight reads serve more rows), 32 on a device list
// (the first round's leftovers, a few thousand pairs: more workgroups, each
// with a shorter chain of tiles; measured 14 us faster there).
constexpr int kActLd = 256 + 8;      // LDS row of one pair's activations (bf16)
constexpr int kOutLd = 64 + 4;       // LDS row of one pair's outputs (FP32, d_out <= 64)

template <int kFRows>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_fused(FusedMlpArgs a) {
  constexpr int kFRT = kFRows / 16;    // row tiles
  __shared__ __align__(16) uint16_t act[kFRows * kActLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (a.np_dev) {
    const int64_t n = (int64_t)*a.np_dev;
    if (n < a.np) a.np = n;
  }
  // tiles of 128 pairs, strided over the grid (the same for every thread of
  // the workgroup, so the barriers below are reached by all or none)
  for (int64_t row0 = (int64_t)blockIdx.x * kFRows; row0 < a.np; row0 += (int64_t)gridDim.x * kFRows) {
  __syncthreads();   // the previous tile's outputs have been copied out of the LDS
  // features of the 128 pairs (rows of X, stride kp[0]; zero rows past the end)
  {
    const int c8 = a.kp[0] / 8;
    for (int q = tid; q < kFRows * c8; q += 256) {
      const int i = q / c8, c = (q % c8) * 8;
      const int64_t w = row0 + i;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (w < a.np) v = *reinterpret_cast<const uint4*>(a.X + w * a.kp[0] + c);
      *reinterpret_cast<uint4*>(&act[i * kActLd + c]) = v;
    }
  }
  __syncthreads();
  const int mrow = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll 1
  for (int l = 0; l < 4; ++l) {
    const int K = a.kp[l], nout = a.nout[l];
    const int nt = (nout + 15) >> 4;             // column tiles of the layer
    const int j0 = 4 * wave;                     // this wave's first column tile
    const bool on = j0 < nt;
    const uint16_t* W = a.wi + a.oWi[l];
    f32x4_t acc[kFRT][4];
#pragma unroll
    for (int i = 0; i < kFRT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    if (on) {
      // B fragment of column tile j0 + j at K slice k0: weight row 16 (j0 + j)
      // + lane % 16, k = k0 + 8 (lane / 16) .. + 7.  Loaded unconditionally
      // (the rows are padded to whole tiles; a tile past the layer's last
      // reads its last row, a slice past K the last slice: both unused)
      const int npad = (nout + 15) & ~15;
      auto loadB = [&](int k0, bf16x8_t (&f)[4]) {
        const int kc = k0 < K ? k0 : K - 32;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = min(16 * (j0 + j) + mrow, npad - 1);
          f[j] = *reinterpret_cast<const bf16x8_t*>(W + (int64_t)n * K + kc + kq);
        }
      };
      bf16x8_t b0[4], b1[4], b2[4];
      loadB(0, b0);
      loadB(32, b1);
      loadB(64, b2);
#pragma unroll 1
      for (int k0 = 0; k0 < K; k0 += 32) {
        // the slice's eight A fragments first, then its 32 MFMAs
        bf16x8_t af[kFRT];
#pragma unroll
        for (int i = 0; i < kFRT; ++i)
          af[i] = *reinterpret_cast<const bf16x8_t*>(&act[(16 * i + mrow) * kActLd + k0 + kq]);
#pragma unroll
        for (int i = 0; i < kFRT; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], b0[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          b0[j] = b1[j];
          b1[j] = b2[j];
        }
        loadB(k0 + 96, b2);
      }
    }
    __syncthreads();   // every wave is done reading this layer's input
    // epilogue: lane holds rows 16 i + 4 (lane / 16) + v, column 16 (j0 + j) +
    // lane % 16; each column is written through one base address with the
    // rows as constant offsets.  Hidden layers: bf16 over the input; the last
    // layer: FP32 rows of kOutLd through the same LDS, then copied out
    const float* bias = a.w32 + a.ob[l];
    if (l < 3) {
      if (on) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = 16 * (j0 + j) + mrow;
          if (j0 + j >= nt || n >= nout) continue;
          const float bn = bias[n];
          uint16_t* base = act + 4 * (lane >> 4) * kActLd + n;
#pragma unroll
          for (int i = 0; i < kFRT; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) base[(16 * i + v) * kActLd] = bf16_rne(fmaxf(acc[i][j][v] + bn, 0.f));
        }
      }
      __syncthreads();   // the next layer reads these outputs
    } else {
      float* of = reinterpret_cast<float*>(act);
      if (on) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = 16 * (j0 + j) + mrow;
          if (j0 + j >= nt || n >= nout) continue;
          const float bn = bias[n];
          float* base = of + 4 * (lane >> 4) * kOutLd + n;
#pragma unroll
          for (int i = 0; i < kFRT; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) base[(16 * i + v) * kOutLd] = acc[i][j][v] + bn;
        }
      }
      __syncthreads();
      for (int q = tid; q < kFRows * nout; q += 256) {
        const int r = q / nout, c = q - r * nout;
        const int64_t w = row0 + r;
        if (w < a.np) a.out[w * nout + c] = of[r * kOutLd + c];
      }
    }
  }
  }
}

// Training labels: the real roots found by the companion solve, in the
// canonical frame (theta + canon, wrapped to [0, 2 pi)), up to Rmax per pair.
__global__ __launch_bounds__(64) void k_labels(const double* rec, int H, int64_t np, float* roots, int* nroots,
                                               int Rmax) {
  const RecLayout RL(H);
  const int lane = threadIdx.x & 63;
  for (int64_t w = blockIdx.x; w < np; w += gridDim.x) {
    const double* R = rec + w * (int64_t)RL.stride;
    const int st = (int)R[RL.meta + M_STATUS];
    // candidates c = lane and lane + 64 (degree D > 64); real ones in order of c
    bool real[2] = {false, false};
    double th[2] = {0.0, 0.0};
    if (st == ST_OK) {
      const unsigned lo = (unsigned)R[RL.meta + M_REAL_LO], hi = (unsigned)R[RL.meta + M_REAL_HI];
      const unsigned long long msk = ((unsigned long long)hi << 32) | lo;
      const unsigned x = RL.D > 64 ? (unsigned)R[RL.meta + M_REAL_X] : 0u;
      for (int sl = 0; sl < 2; ++sl) {
        const int cidx = lane + 64 * sl;
        if (cidx >= RL.D) continue;
        real[sl] = sl == 0 ? ((msk >> lane) & 1ull) != 0ull : lane < 32 && ((x >> lane) & 1u) != 0u;
        double v = R[RL.cand + cidx] + R[RL.meta + M_CANON];
        v = fmod(v, kTwoPi);
        th[sl] = v < 0.0 ? v + kTwoPi : v;
      }
    }
    const unsigned long long m0 = __ballot(real[0]), m1 = __ballot(real[1]);
    const unsigned long long below = (1ull << lane) - 1ull;
    const int pos0 = __popcll(m0 & below), pos1 = __popcll(m0) + __popcll(m1 & below);
    if (real[0] && pos0 < Rmax) roots[w * Rmax + pos0] = (float)th[0];
    if (real[1] && pos1 < Rmax) roots[w * Rmax + pos1] = (float)th[1];
    const int nr = __popcll(m0) + __popcll(m1);
    if (lane == 0) nroots[w] = nr < Rmax ? nr : Rmax;
  }
}

// ------------------------------------------------------------ launchers

hipError_t launch_dense(const uint16_t* A, int64_t lda, const uint16_t* W, int ldw, const float* bias, int64_t M,
                        int N, int Kp, int relu, uint16_t* Yb, float* Yf, int64_t ldy, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  DenseArgs d{A, lda, W, ldw, bias, M, N, Kp, relu, Yb, Yf, ldy};
  dim3 grid((unsigned)((M + 64 * kDRW - 1) / (64 * kDRW)), (unsigned)((N + kDC - 1) / kDC));
  hipLaunchKernelGGL(k_dense_bf16<kDRW>, grid, dim3(256 * kDRW), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.M + kGT - 1) / kGT), (unsigned)((g.N + kGT - 1) / kGT));
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int64_t M, int N, int64_t ld, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, G, M, N, ld, out);
  return hipGetLastError();
}

hipError_t launch_chamfer(const float* out, int64_t B, int Kseeds, const float* roots, const int* nroots, int R,
                          float lam, float* loss_b, float* dout, uint16_t* dout_bf, hipStream_t st) {
  hipLaunchKernelGGL(k_chamfer, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, out, B, Kseeds, roots,
                     nroots, R, lam, loss_b, dout, dout_bf);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, uint16_t* wb, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, wb, g, m, v, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

bool mlp_fused_ok(const int* nin, const int* nout) {
  if (((nin[0] + 31) & ~31) > 256 || nout[3] < 1 || nout[3] > 64) return false;
  for (int l = 0; l < 3; ++l)
    if (nout[l] % 32 != 0 || nout[l] > 256) return false;
  return nin[1] == nout[0] && nin[2] == nout[1] && nin[3] == nout[2];
}

// grid: at most max_blocks workgroups, each taking every max_blocks-th tile
// of 128 pairs (32 on a device list)
// `done` (nullable): an event the launch records at the kernel's end.
hipError_t launch_mlp_fused(const FusedMlpArgs& fa, hipStream_t st, int max_blocks, hipEvent_t done) {
  if (fa.np <= 0) return done ? hipEventRecord(done, st) : hipSuccess;
  const int rows = fa.np_dev ? 32 : 128;
  int64_t blocks = (fa.np + rows - 1) / rows;
  if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
  if (fa.np_dev)
    hipExtLaunchKernelGGL(k_mlp_fused<32>, dim3((unsigned)blocks), dim3(256), 0, st, nullptr, done, 0, fa);
  else
    hipExtLaunchKernelGGL(k_mlp_fused<128>, dim3((unsigned)blocks), dim3(256), 0, st, nullptr, done, 0, fa);
  return hipGetLastError();
}

// Features of pairs [0, np) of the chunk (row i = pair i), or, with a list,
// of the pairs list[0 .. *list_count) (row i = pair list[i]; np bounds the
// grid only).
hipError_t launch_features(double* rec, int H, int64_t np, uint16_t* X, int64_t ldx, int waves, hipStream_t st,
                           const int64_t* list, const unsigned* list_count) {
  if (6 * H - 2 < 64) {
    const int w2 = (int)std::max<int64_t>(1, std::min<int64_t>(waves, (np + 1) / 2));
    hipLaunchKernelGGL(k_features2, dim3((unsigned)w2), dim3(64), 0, st, rec, H, np, X, ldx, list, list_count);
  } else {
    hipLaunchKernelGGL(k_features, dim3((unsigned)waves), dim3(64), 0, st, rec, H, np, X, ldx, list, list_count);
  }
  return hipGetLastError();
}

hipError_t launch_labels(const double* rec, int H, int64_t np, float* roots, int* nroots, int Rmax, int waves,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_labels, dim3((unsigned)waves), dim3(64), 0, st, rec, H, np, roots, nroots, Rmax);
  return hipGetLastError();
}

}  // namespace ftp
