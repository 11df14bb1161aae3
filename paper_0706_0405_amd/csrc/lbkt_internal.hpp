// Internal interface between the translation units of liblbkt.so (not part of
// the C ABI): the host-side constant builder and the error recorder of lbkt.hip.
#pragma once

#include <string>

#include "../../include/lbkt.h"
#include "kt_site.hpp"

// Fill the per-launch constants of the step for a validated grid.
void lbkt_build_consts(const lb_grid* g, lbkt::KTConsts* K);

// Record msg as the calling thread's lb_last_error() text and return s.
lb_status lbkt_fail(lb_status s, const std::string& msg);
