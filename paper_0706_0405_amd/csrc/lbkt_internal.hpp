// Internal interface between the translation units of liblbkt.so (not part of
// the C ABI): the host-side constant builder and the error recorder of lbkt.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

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
lb_status lbkt_invariants_args(const lb_grid* g, lb_prec prec, const void* f, const double* out4);
lb_status lbkt_launch_invariants(const lbkt::KTConsts& K, lb_prec prec, const void* f, int rows_per_block,
                                 int nblocks, double* part, double* out4, hipStream_t st);
