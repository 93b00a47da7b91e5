// nyx_launch.h -- host-side launchers of the kernels in nyx_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "nyx_types.h"

namespace nyx {

hipError_t launch_max_label(const ImgDesc *imgs, int n_images, uint32_t *out, hipStream_t st);
hipError_t launch_label_collect(const ImgDesc *imgs, int n_images, uint64_t max_vox, uint64_t *list, uint32_t cap,
                                uint32_t *count, hipStream_t st);
hipError_t launch_reset(const StepArgs &a, uint32_t n_counters, hipStream_t st);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st);
hipError_t launch_zero_split(const StepArgs &a, hipStream_t st);
hipError_t launch_scan(const StepArgs &a, hipStream_t st);
hipError_t launch_compact(const StepArgs &a, uint32_t roi_lo, uint32_t roi_hi, hipStream_t st);
hipError_t launch_bin_image(const StepArgs &a, uint16_t *bins, uint64_t total_vox, const uint64_t *img_vox_base,
                            hipStream_t st);
hipError_t launch_batch(const StepArgs &a, uint32_t grid, uint32_t block, uint32_t direct_roi, hipStream_t st);
hipError_t get_batch_attributes(int mode, int fp64, int ns, uint32_t block, hipFuncAttributes *attr);
hipError_t batch_occupancy(int mode, int fp64, int ns, uint32_t block, uint32_t lds_bytes, int *blocks_per_cu);
hipError_t launch_band(const StepArgs &a, uint32_t grid, hipStream_t st);
hipError_t launch_split_finalize(const StepArgs &a, hipStream_t st);
hipError_t launch_features(const StepArgs &a, const DirSums *ds, const DirSumsY *dsy, uint32_t n_cap,
                           const uint32_t *n_ptr, hipStream_t st);
hipError_t launch_coo_count(const StepArgs &a, uint32_t n_slots, uint64_t *counts, hipStream_t st);
hipError_t launch_coo_emit(const StepArgs &a, uint32_t n_slots, const uint64_t *offsets, uint64_t *keys,
                           uint64_t *vals, hipStream_t st);
hipError_t launch_coo_features(const StepArgs &a, const uint64_t *keys, const uint64_t *vals, uint64_t nnz,
                               uint32_t n_rois, uint64_t *seg, DirSums *sums, DirSumsY *sums_y, hipStream_t st);
hipError_t launch_intensity(const StepArgs &a, uint32_t grid, int fp64, void *table, uint32_t table_rows,
                            hipStream_t st);
uint32_t neighbourhood_lds_bytes(uint32_t ng, int any_volume);
hipError_t launch_neighbourhood(const StepArgs &a, uint32_t grid, int fp64, uint32_t alpha, int any_volume,
                                void *table, uint32_t table_rows, hipStream_t st);

}  // namespace nyx
