// kernels.hpp -- launchers of the sweep kernels (internal to libsweep).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_math.hpp"

namespace sweep {

struct InitialNormal {
    int enabled;
    double v[3];
};

int frame_chunk_size();

// Default knot vector (clamped uniform, or periodic U_k = k) written on the device.
hipError_t launch_fill_knots(double* U, int n, int p, int closed, hipStream_t st);

hipError_t launch_path_samples(const DCurve& path, int n_u, double* smp, int* chunk_lv, double* fallback_t,
                               hipStream_t st);
template <class T>
hipError_t launch_profile_table(const DCurve& prof, int n_v, T* tab, hipStream_t st);
template <class F, class T>
hipError_t launch_frame(const double* smp, int n_u, const int* chunk_lv, const double* fallback_t,
                        InitialNormal n0, int reorth, F* agg, F* r_in, T* rows, hipStream_t st);

// Surface write of one sweep from its row table (16 values per u-row) and
// profile table (8 values per v-sample).
struct SurfaceConfig {
    int kind;           // 0: column-stationary vector stores, 1: linear dword stores
    int rows_per_block; // kind 0
    int tile_vertices;  // kind 1: vertices per block-tile (multiple of 256)
    int grid;           // kind 1: persistent grid size (0 = one block per tile)
    int nontemporal;    // nontemporal stores
};

template <class T>
hipError_t launch_surface(const T* rows, const T* prof, int n_u, int n_v, T* pos, T* nrm,
                          const SurfaceConfig& cfg, hipStream_t st);

bool surface_cols_supported(int n_v, const void* pos, const void* nrm, size_t elem);

}  // namespace sweep
