// Stencil launch configuration cache (filled by the autotuner, read by every driver).
#pragma once

#include <string>

#include "rmh_internal.h"

namespace rmh {

// purpose: an rmh_purpose value (RMH_PURPOSE_ANY .. RMH_PURPOSE_HEATBATH)
HopConfig tune_hop(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose);
void tune_store(const Geom& g, int32_t dtype, int32_t n_rhs, int32_t purpose, const HopConfig& cfg, double ms);
void tune_clear();
// why a configuration is invalid for dtype, or nullptr
const char* hop_config_error(const HopConfig& cfg, int32_t dtype);
// the cache as a JSON file stamped with the device architecture and HIP runtime version:
// 0 on success, -1 when the file cannot be written / read, -2 (load) when it is malformed or holds an
// invalid entry; a file of another architecture or runtime loads nothing
int tune_save_file(const char* path, const std::string& arch, int32_t runtime, int32_t* n_saved);
int tune_load_file(const char* path, const std::string& arch, int32_t runtime, int32_t* n_loaded);

}  // namespace rmh
