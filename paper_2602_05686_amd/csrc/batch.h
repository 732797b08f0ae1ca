// Batched solve-path launches: one launch runs the same step for many
// hierarchies.  A launch covers `nseg` segments; segment j owns the blocks
// [starts[j], starts[j+1]) of the launch (starts[nseg] = total) and its own
// argument record args[j].  Inside a segment every block does exactly what
// the one-hierarchy launch does for the same block index, so each
// hierarchy's results are independent of the batch it is launched in.
// `args` and `starts` are device pointers.
#pragma once

#include "solve_device.h"

namespace matamg {

// streaming SpMV of mode `mode` (StreamMode) with `group` threads per row
// (1 or 8); segment j has the matrix's row-block count.  Precision: float
// or double records.
template <typename T>
void stream_batch(int mode, bool has_dot, int group, const SArgs<T>* args, const int* starts, int nseg, int total,
                  hipStream_t s);
// segment j has vec_grid(n_j) blocks
template <typename T>
void smooth_first_batch(const SmoothFirstArgs<T>* args, const int* starts, int nseg, int total, hipStream_t s);
void cg_direction_batch(const CgDirArgs* args, const int* starts, int nseg, int total, hipStream_t s);
void cg_update_batch(const CgUpdArgs* args, const int* starts, int nseg, int total, hipStream_t s);
// one block per record
void finish_batch(const FinishArgs* args, int nseg, hipStream_t s);
// segment j has gemv_grid(n_j) blocks
template <typename T>
void gemv_batch(const GemvArgs<T>* args, const int* starts, int nseg, int total, hipStream_t s);

}  // namespace matamg
