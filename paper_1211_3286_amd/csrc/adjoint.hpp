// Tape (checkpoints of g) and the reverse sweep behind rlb_grad.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rlb.h"
#include "internal.hpp"

namespace rlb {

// Byte offsets inside the tape region of the workspace.
struct TapeLayout {
  size_t gbytes = 0;      // one g state: 19 planes of cs elements
  int n_ckpt = 0;         // checkpoints at steps 0, K, 2K, ...
  int K = 0;
  size_t off_ckpt = 0;    // n_ckpt g states
  size_t off_seg = 0;     // 2K g states: the segment being reversed, the next recomputed
  size_t off_adj = 0;     // two adjoint g buffers
  size_t off_fields = 0;  // eps0, u0 (4 * ncells doubles)
  size_t off_tparts = 0;  // per-block tau-gradient partials (max_parts * 5 doubles)
  size_t total = 0;
  int max_parts = 0;
};

TapeLayout tape_layout(int nx, int ny, int nz, int64_t cs, size_t esz, int K, int tape_steps,
                       int max_parts);

struct Tape {
  char* base = nullptr;
  TapeLayout L;
  int precision = 0;
  int64_t ncells = 0, cs = 0;
  // the reverse sweep's kernel chain, instantiated for graph_steps steps
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int64_t graph_steps = -1;
};

rlb_status tape_init(Tape& t, const TapeLayout& L, char* base, int precision, int64_t ncells,
                     int64_t cs, int K, int tape_steps, const double* n0, const double* eps0,
                     const double* u0, const void* state, hipStream_t s);
rlb_status tape_checkpoint(Tape& t, int64_t idx, const void* state, hipStream_t s);

struct GradContext {
  int precision;
  int64_t ncells, cs;
  MemberDesc desc;        // geometry, rates and reference of the (single) lattice
  int64_t steps;          // forward steps taken since rlb_init
  bool tau_q_tied;        // ghost rows relax with tau_v
  const void* state;      // current population buffer (38 planes)
  double* stage;          // 8 * ncells doubles of staging
  double* sums_out;       // 5 doubles of device scratch
  hipStream_t stream;
};

rlb_status tape_grad(Tape& t, const GradContext& c, const double* dL_du, const double* dL_deps,
                     double dL_dtau[3], double* dL_deps0, double* dL_du0, int io_on_device);
void tape_release(Tape& t);  // also destroys the kept graph

}  // namespace rlb
