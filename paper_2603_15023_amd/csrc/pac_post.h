// Host entry points of the vector-lifted expressions (k_post.hip) and of
// pac_noised over given world vectors (k_finalize.hip).
#pragma once
#include "pac_internal.h"

namespace pac {

// A validated postfix program, passed to the kernel by value.
struct LiftProg {
  const double *in[PAC_LIFT_MAX_INPUTS];
  uint32_t scalar;  // bit k: input k is [G], broadcast over the worlds
  int32_t n_ops;
  int8_t op[PAC_LIFT_MAX_OPS];
  int8_t arg[PAC_LIFT_MAX_OPS];
  double val[PAC_LIFT_MAX_OPS];
};

// pac_select_cmp through a table of the comparison's words for every group and
// integer value in [lo, lo + R) (table: [n_groups][R][W] words of scratch);
// rows with other values take the row-wise form.
hipError_t launch_select_table(const LaunchEnv &env, const DevInput &in, const double *wv, int op, double scale,
                               double offset, int64_t lo, int32_t R, uint64_t *table, uint64_t *out);
hipError_t launch_lift(const LaunchEnv &env, const LiftProg &prog, int64_t G, int m, double *out);
hipError_t launch_noised(const LaunchEnv &env, const double *wv, const int64_t *cell_rows, int64_t first_cell,
                         const FinParams &fp, double *out_val, uint8_t *out_is_null, uint32_t *out_flags,
                         double *posterior, void *scratch);

}  // namespace pac
