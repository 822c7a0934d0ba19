// Work schedules of the batched and 4D launches (host code, no device calls).
//
// A launch of the persistent kernels runs a list of work items (field, unit
// range) split over its workgroups: items are cut from each field so that no
// workgroup's packed LDS bins see more cells between drains than the bin
// layout allows, and dealt to workgroups largest first onto the least loaded.
#pragma once

#include <cstdint>
#include <vector>

#include "ecc_internal.h"

namespace ecc {

struct SchedField {
    int32_t slot;  // descriptor index the items refer to
    int64_t h, w;
    int64_t d = 1;
};

struct TileShape {
    int tx, ty, tz;
};

// deal items (costs given, plus per_item each) to `grid` workgroups, largest
// first onto the least loaded; out: items grouped by workgroup, first[grid + 1]
void deal_items(const std::vector<BatchItem> &items, const std::vector<int64_t> &cost, int64_t per_item, int grid,
                std::vector<BatchItem> &sorted, std::vector<int32_t> &first);

// 2D: items of (strip, row) units; returns the grid, n_items per field
int schedule_batch_2d(int n_cu, int dtype, int lm, int max_L, const std::vector<SchedField> &fields,
                      int item_cells, int wg_per_cu, std::vector<BatchItem> &sorted, std::vector<int32_t> &first,
                      std::vector<int32_t> &n_items);

// tile shape of a batched (or 4D-slice) volume of d x h x w voxels
TileShape tile_shape_3d(int64_t d, int64_t h, int64_t w);

// 3D: items of whole tiles of each volume's tile shape
int schedule_batch_3d(int n_cu, int max_L, const std::vector<SchedField> &fields, int item_cells, int wg_per_cu,
                      std::vector<BatchItem> &sorted, std::vector<int32_t> &first, std::vector<int32_t> &n_items);

// 4D: items of whole tiles of the n_vol virtual volumes (slices and images)
// of d x h x w voxels; returns the grid
int schedule_4d(int n_cu, int L, int64_t n_vol, int64_t d, int64_t h, int64_t w, const TileShape &ts,
                std::vector<BatchItem> &sorted, std::vector<int32_t> &first);

// LDS bytes of the dynamic part of a workgroup of each kernel
size_t lds_bytes_batch_2d(int lm, int max_L);
size_t lds_bytes_batch_3d(int max_L);
size_t lds_bytes_4d(int L);

}  // namespace ecc
