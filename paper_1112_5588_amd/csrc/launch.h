// Kernel launchers shared between the HIP translation units of libpjds.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.h"

namespace pjds {
// Events armed on the calling thread by pjds_time_next_launch; taking them disarms the hook.
struct LaunchEvents {
    hipEvent_t start, stop;
};
LaunchEvents take_launch_events();

// Launch of an entry point's main kernel.  When the measurement hook is armed, the kernel's
// own dispatch records the armed events at its start and end; otherwise this is an ordinary
// launch (hipExtLaunchKernel with no events).  Errors are left for hipGetLastError.
template <class F, class... A>
inline void launch_main(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, A... a) {
    const LaunchEvents ev = take_launch_events();
    hipExtLaunchKernelGGL(kernel, grid, block, uint32_t(lds), s, ev.start, ev.stop, 0u, a...);
}

// Kernel launchers shared between translation units (spmv.hip).  The caller validates.
// Sizes, dtype and block height of a pJDS matrix usable by the single-vector product.
int check_product_info(const pjds_info *info, int32_t dtype);
int check_xlds(const pjds_info &in, int32_t dtype, int32_t x_halo, int32_t tile_rows);
// Workgroups (row tiles) of the staged product: one per tile, the tile index = its rows / tile.
int64_t xlds_tiles(const pjds_info &in, int32_t tile_rows);
// ea.dot_partial needs PJDS_TWO_ROWS (the two-rows kernel computes it).
void launch_xlds(const pjds_info &in, const int32_t *d_row_len, const int64_t *d_offsets, const int32_t *d_col_p,
                 const void *d_val_p, const int32_t *d_perm, int32_t dtype, const void *d_x, void *d_y,
                 int32_t x_halo, int32_t tile_rows, const EpiArgs &ea, uint32_t flags, hipStream_t s);
void launch_spmv_epi(const pjds_info &in, const int32_t *d_row_len, const int64_t *d_offsets,
                     const int32_t *d_col_p, const void *d_val_p, const int32_t *d_sched, void *d_work,
                     int32_t dtype, const void *d_x, void *d_y, const EpiArgs &ea, uint32_t flags,
                     hipStream_t s);
}  // namespace pjds

