// gm_internal.hpp -- host-side declarations shared by the libgm translation
// units (options, workspace layout, run results).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>

#include "../../include/gm.h"
#include "gm_common.hpp"

namespace gm {

struct Options {
  int init_log2 = 12;        // initial partition 2^(d*floor(init_log2/d)) cells
  int64_t max_iters = 10000; // iteration budget
  int graph_iters = 0;       // iterations per graph replay (0 = direct launches)
  int lanes_per_region = 0;  // rule-kernel mapping (0 = automatic)
  int timing = 0;            // per-phase hipEvent timing
  int log = 0;               // per-iteration log to stderr
  int rule = 0;              // 0 Genz-Malik degree 7, 1 tensor-product Gauss-Kronrod
                             // (d <= 6), 2 degree-9 fully symmetric rule
  int err_model = 0;         // degree-9 rule: 0 |Q9 - Q7|, 1 null-rule ratio test
  int prune = 0;             // memory-pressure pruning instead of stopping at capacity
};

// Byte offsets of the device buffers of one run inside the workspace.
struct Layout {
  size_t C[2], H[2], L[2], PAX[2];
  size_t Q, ERR, AXIS, FLAG;
  size_t TK, TOFF, TQ, TE;
  size_t PART, ST, HIST;
  size_t total;
};

struct RunResult {
  double I = 0, E = 0;
  int status = 0;
  int64_t final_n = 0;
  int64_t final_npar = 0;  // parent records behind the final set when it is split
  int final_split = 0;
  int buf = 0;
  int64_t leaf_count = 0;
  char* base = nullptr;
  Layout lay{};
  int64_t cap = 0;
  double vol_omega = 1.0;
};

Options& options();
Layout make_layout(int d, int64_t cap);
size_t align256(size_t x);
int acquire_workspace(size_t bytes, char** base);
void fill_consts(int d, RuleConsts& K);
void fill_params(int fam, int d, const double* params, DevParams& P);
int validate(int fam, const double* params, int d, const double* lo, const double* hi,
             double rel_tol, double abs_tol);
hipError_t launch_rule(int d, int fam, int log2l, const RuleArgs& a, int grid, hipStream_t s);
// Rule-kernel mapping for n regions of dimension d: -1 = one lane per region,
// else log2 of the lanes per region.
int choose_mapping(int d, int64_t n);
RuleKernelFn rule_kernel(int d, int fam, int log2l, bool batch);
// Degree-9 rule kernel of (d, family): single-store or batch-store variant;
// `wide`: the single-store kernel with 2^rule9_log2l_wide(d) lanes per region.
RuleKernelFn r9_kernel(int d, int fam, bool batch, bool wide = false);
// Gauss-Kronrod rule kernel of (d, family), d <= kGkMaxDim.
RuleKernelFn gk_kernel(int d, int fam, bool batch);
// Nodes of the rule the options select.
int64_t nodes_per_region(int d);
bool mapping_allowed(int d, int log2l);
int rule_grid(int log2l, int64_t n, int d);
// fixed_base: when not null, the run's device buffers are laid out from it
// (the no-allocation entry point's fixed scratch, already checked to be large
// enough) and the run allocates nothing: no workspace, no pinned status copy
// (an existing one is used), no timing events.
int run_adaptive(int fam, const double* params, int d, const double* lo, const double* hi,
                 double rel_tol, double abs_tol, int64_t max_regions, hipStream_t s,
                 bool keep_leaves, RunResult* out, char* fixed_base = nullptr);
size_t batch_layout_bytes(int dmax, int64_t cap);

// Process-wide lock serialising every C ABI call.
std::mutex& api_mutex();
// Record a HIP error for gm_status_string(GM_EHIP) and return GM_EHIP.
int record_hip_error(hipError_t e);

// Bounds checks of a GM_CHECK build (gm_common.hpp): called after a call's
// device work has finished, polls every translation unit's check record and
// returns GM_EHIP, with the first violation as gm_status_string(GM_EHIP), if
// any unit counted one; otherwise (and always without GM_CHECK) returns rc.
int check_bounds(int rc);
#ifdef GM_CHECK
#define GM_DECLARE_POLL_F(name)                                                          \
  int gm_check_poll_##name##_f1(CheckRec*); int gm_check_poll_##name##_f2(CheckRec*);    \
  int gm_check_poll_##name##_f3(CheckRec*); int gm_check_poll_##name##_f4(CheckRec*);    \
  int gm_check_poll_##name##_f5(CheckRec*); int gm_check_poll_##name##_f6(CheckRec*);    \
  int gm_check_poll_##name##_f7(CheckRec*);
int gm_check_poll_api(CheckRec*);
int gm_check_poll_batch(CheckRec*);
int gm_check_poll_grad(CheckRec*);
GM_DECLARE_POLL_F(rule)
GM_DECLARE_POLL_F(rule9)
GM_DECLARE_POLL_F(adjoint)
GM_DECLARE_POLL_F(gk)
#undef GM_DECLARE_POLL_F
#endif

// The retired-leaf store of the last gradient-mode forward run (SoA).
struct LeafView {
  const double* C;
  const double* H;
  const uint16_t* L;
  int64_t cap;
};
LeafView leaf_view();

// Statistics of the last call (gm_last_stats).
void stats_reset();
gm_stats& stats_ref();

}  // namespace gm
