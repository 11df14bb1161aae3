// Internal interface between the translation units of liblbkt.so (not part of
// the C ABI): the host-side constant builder and the error recorder of lbkt.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbkt.h"
#include "kt_site.hpp"

// Fill the per-launch constants of the step for a validated grid.
void lbkt_build_consts(const lb_grid* g, lbkt::KTConsts* K);

// Record msg as the calling thread's lb_last_error() text and return s.
lb_status lbkt_fail(lb_status s, const std::string& msg);

// lb_invariants: partial sums of at most LBKT_INV_MAX_PARTS blocks of rows, then a
// final sum (the partition, the argument checks and the two kernel launches).
constexpr int LBKT_INV_MAX_PARTS = 4096;
void lbkt_inv_partition(const lb_grid* g, int* rows_per_block, int* nblocks);
lb_status lbkt_invariants_args(const lb_grid* g, int32_t prec, const void* f, const double* out4);
lb_status lbkt_launch_invariants(const lbkt::KTConsts& K, lb_prec prec, const void* f, int rows_per_block,
                                 int nblocks, double* part, double* out4, hipStream_t st);

// Moving-shock edge `edge` (2: y-, 3: y+) at time index `step`: the number of its
// ghost cells whose centre lies behind the shock (0 for other edge kinds).
int lbkt_shock_cells(const lb_grid* g, int edge, int64_t step);

// Default launch shape of the two-step pass for an nx x ny grid.
void lbkt_default_tile2(int nx, int ny, lb_prec prec, int* block_x, int* rows);

// One work item of the batched kernels: a column strip of one problem.
struct LbktWorkItem {
  int32_t prob;
  int32_t strip;
};

// Work lists of a batch for block_x threads per item: one-step items (strips of
// block_x columns) and two-step items (strips of block_x / 64 wavefronts of 60
// columns), problems longest first, the two-step list dealt to the XCDs in runs.
void lbkt_plan_batch(const lb_grid* grids, int nprob, int block_x, std::vector<LbktWorkItem>* items,
                     std::vector<LbktWorkItem>* items2);

// Work list of the deep passes (depth = 4, 6 or 8 steps per pass): strips of
// 64 - 2 * depth output columns per wavefront, ordered and dealt as items2.
void lbkt_plan_batch_deep(const lb_grid* grids, int nprob, int block_x, int depth,
                          std::vector<LbktWorkItem>* items);

// Neighbours of each two-step item (the items whose columns its wavefronts read:
// the strips left and right of it in its problem, wrapped for a periodic x axis;
// -1 for none or itself).
void lbkt_batch_neighbours(const lb_grid* grids, const std::vector<LbktWorkItem>& items2, int block_x,
                           std::vector<int>* left, std::vector<int>* right);
