// Argument blocks of the per-frequency kernels that the host runtime
// launches, shared by the kernels' sources and ftp_capi.hip (one definition).
#pragma once

#include "ftp_internal.h"

namespace ftp {

// Newton + Sturm (first round): pairs [0, np) of a record chunk.
struct LearnArgs {
  double* rec;
  int64_t np;
  const float* seeds_out;   // network output, np x 4H (u, v pairs); nullptr = evenly spaced starts
  int64_t* fb_list;         // pairs the round leaves unconfirmed
  unsigned int* fb_count;
  unsigned flags;           // bit 0: forced fallback (every pair to the list); bit 1: 2H starts only
  unsigned* queue;          // work counter (zeroed), or nullptr for grid striding
};

// Second Newton round over the first round's list (k_newton_retry).
struct RetryArgs {
  double* rec;
  int H;
  const int64_t* list;       // first-round fallback list
  const unsigned* count;     // its length
  const float* seeds;        // nullable: network output rows in list order
  int64_t* out_list;         // pairs left to the Aberth tier
  unsigned* out_count;
  SolveCounters* counters;
};

// Aberth tier (or the Aberth solver over every pair).
struct AberthArgs {
  double* rec;
  int64_t np;
  const int64_t* list;       // pairs to solve; nullptr = every pair of the chunk
  const unsigned* count;     // length of `list`
  int64_t* qr_list;          // pairs left to the companion-matrix solve
  unsigned* qr_count;
  SolveCounters* counters;
  int H;
  double mark;               // M_FALLBACK value written for pairs sent on
  unsigned flags;            // bit 0: send every pair on (companion solve only)
  unsigned* queue;           // work counter (zeroed), or nullptr for grid striding
};

// The four network layers in one kernel (k_mlp_fused).
struct FusedMlpArgs {
  const uint16_t* X;     // np x kp[0] bf16 features (zero padded)
  int64_t np;
  const uint16_t* wi;    // padded bf16 weights, layer l at wi + oWi[l], rows of kp[l]
  const float* w32;      // FP32 parameters (biases at w32 + ob[l])
  int64_t oWi[4], ob[4];
  int kp[4], nout[4];
  float* out;            // np x nout[3]
  const unsigned* np_dev;   // nullable: rows past *np_dev (on the device) are skipped
};

}  // namespace ftp
