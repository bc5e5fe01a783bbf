// Host-side launchers of the gfx950 kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.hpp"

namespace lbmib {

// Sweep tilings: threads along x, thread rows per block, lattice rows per thread.
struct Tiling {
    int tx, ty, rpt, nontemporal;
};
constexpr int kNumTilings = 20;
extern const Tiling kTilings[kNumTilings];

// Entries sorted in LDS when a plan is rebuilt on the device (16 per marker).
constexpr int kMaxDynEntries = 8192;
constexpr int kMaxGroupMarkers = 4096;
constexpr int kMaxColors = 32;  // colour classes of a band spread without conflicts

// Static device staging (lbm_fields_noalloc): 8 MiB per device.
constexpr size_t kStaticScratchDoubles = size_t(1) << 20;
constexpr int kMaxDevices = 64;
// Device address of this device's staging array (taken once per device).
hipError_t static_scratch(double** out);

// All launchers enqueue on `stream`.  `parity` >= 0 forces the AA state the
// step starts from; -1 reads it from each simulation's descriptor (batches).
// Counts come from `hdr` when it is non-null (graph-captured batches),
// otherwise from the explicit count arguments.
// mrt: some simulation of the launch uses the MRT collision.
hipError_t launch_sweep(bool f64, bool mrt, int tiling, const SimDev* sims, const int4* tiles,
                        const BatchHeader* hdr, int ntiles, int grid, int parity, hipStream_t stream);
hipError_t launch_boundary(bool f64, const SimDev* sims, const int2* items, const BatchHeader* hdr,
                           int nitems, int grid, int parity, hipStream_t stream);
// max_markers: the largest group's marker count (selects how many markers
// each thread carries; the results do not depend on it).  lean: FP32 groups of
// at most 1280 markers run in the 256-thread kernels that fit beside sweep
// waves (for lanes whose corrections overlap another lane's sweep).
// bc_items (with hdr): the lane's boundary items, applied by the correction
// workgroups after their groups in place of launch_boundary (only when no band
// of the lane comes within three nodes of a non-periodic side).
hipError_t launch_ib(bool f64, int max_markers, const SimDev* sims, GroupDev* groups, const BatchHeader* hdr,
                     int ngroups, int grid, int parity, hipStream_t stream, bool lean = false,
                     const int2* bc_items = nullptr);
// Band kernels over chunks of 256 band nodes (group, first node): apply =
// false gathers the band records of fixed-plan groups before k_ib, apply =
// true spreads the per-marker totals and corrects the populations after it.
hipError_t launch_band(bool f64, bool apply, const SimDev* sims, const GroupDev* groups, const int2* chunks,
                       const BatchHeader* hdr, int nchunks, int grid, int parity, hipStream_t stream);
hipError_t launch_advance(SimDev* sims, const BatchHeader* hdr, int nsims, hipStream_t stream);
// Whether kernels launched on `second` run while one on `first` runs (the two
// streams reach the GPU through different hardware queues).  flags: two ints
// of device memory; synchronises both streams; takes at most about 0.2 ms.
hipError_t streams_run_concurrently(hipStream_t first, hipStream_t second, int* flags, bool* concurrent);
// which k_ib instance launch_ib picks for a largest group of max_markers
int ib_variant(bool f64, int max_markers, bool lean);
// Field and population I/O of one simulation (state `sw` = AA state now).
hipError_t launch_fields(bool f64, const SimDev* sim, int nx, int ny, int sw, double* rho,
                         double* ux, double* uy, hipStream_t stream);
// rows y0 .. y0 + rows - 1 only, written from index 0 of the outputs
hipError_t launch_fields_rows(bool f64, const SimDev* sim, int nx, int y0, int rows, int sw, double* rho,
                              double* ux, double* uy, hipStream_t stream);
hipError_t launch_get_pop(bool f64, const SimDev* sim, int nx, int ny, int sw, double* f,
                          hipStream_t stream);
hipError_t launch_set_pop(bool f64, const SimDev* sim, int nx, int ny, int sw, const double* f,
                          hipStream_t stream);
// Equilibrium of the given FP64 device fields (or of rho0/u0 when the field
// pointers are null).
hipError_t launch_set_eq(bool f64, const SimDev* sim, int nx, int ny, int sw, const double* rho,
                         const double* ux, const double* uy, double rho0, double u0x, double u0y,
                         hipStream_t stream);

}  // namespace lbmib
