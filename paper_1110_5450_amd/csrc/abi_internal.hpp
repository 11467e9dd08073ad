// abi_internal.hpp -- host helpers shared by the ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/sweep.h"
#include "kernels.hpp"

namespace sweep {

sweep_status fail(sweep_status st, const char* fmt, ...);
sweep_status hip_fail(hipError_t e, const char* where);
sweep_status check_curve_meta(int n, int p, int closed, const double* knots, const char* what, bool is_path);
sweep_status check_curve(const sweep_curve* c, const char* what, bool is_path);
sweep_status check_options(const sweep_options* o);
sweep_status check_grid(int n_u, int n_v);
int nbasis(int n, int p, int closed);
int nknots(int n, int p, int closed);
int tile_config_count();
const SurfaceConfig& tile_config(int k);
SurfaceConfig auto_surface_config(int n_u, int n_v, int t64);
bool options_ext(const sweep_options* o);
bool options_single_only(const sweep_options* o);
// Autotuning table (tune_table.hip): best surface configuration per (kind,
// device, shape class of kTuneClassInts integers), -1 if none recorded.
constexpr int kTuneClassInts = 5;
int tune_lookup(const char* kind, const int* cls);
void tune_record(const char* kind, const int* cls, int config, float ms);
int ilog2_ll(long long v);
sweep_status upload_knots(const double* host_knots, int n, int p, double* dst, hipStream_t st);

}  // namespace sweep
