// Stencil launch configuration cache (filled by the autotuner, read by every driver).
#pragma once

#include "rmh_internal.h"

namespace rmh {

// purpose: 0 plain apply, 1 CG working precision, 2 FP64 residuals, 3 moments, 4 filter
HopConfig tune_hop(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose);
void tune_store(const Geom& g, int32_t dtype, int32_t n_rhs, const HopConfig& cfg);
void tune_clear();

}  // namespace rmh
