// Work schedules of the batched and 4D launches (host code).
#include "ecc_schedule.h"

#include <algorithm>
#include <functional>
#include <queue>
#include <utility>

namespace ecc {

size_t lds_bytes_batch_2d(int lm, int max_L) {
    const bool thr = lm == LM_AFFINE || lm == LM_SEARCH;
    return (size_t)(max_L + 2 * kBinOff) * 8 + (thr ? (size_t)(max_L + 3) * 4 : 0);
}

size_t lds_bytes_batch_3d(int max_L) { return (size_t)max_L * 12; }

size_t lds_bytes_4d(int L) { return (size_t)L * 8; }

void deal_items(const std::vector<BatchItem> &items, const std::vector<int64_t> &cost, int64_t per_item, int grid,
                std::vector<BatchItem> &sorted, std::vector<int32_t> &first) {
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    typedef std::pair<int64_t, int> Load;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> pq;
    for (int wg = 0; wg < grid; ++wg) pq.push({0, wg});
    std::vector<std::vector<int>> per_wg(grid);
    for (int i : order) {
        Load l = pq.top();
        pq.pop();
        per_wg[l.second].push_back(i);
        l.first += cost[i] + per_item;  // + a fixed cost per item (drain, ticket)
        pq.push(l);
    }
    sorted.clear();
    sorted.reserve(items.size());
    first.assign(grid + 1, 0);
    for (int wg = 0; wg < grid; ++wg) {
        first[wg] = (int32_t)sorted.size();
        for (int i : per_wg[wg]) sorted.push_back(items[i]);
    }
    first[grid] = (int32_t)sorted.size();
}

// Cut fields into items of at most `item_cells` cells (counted as whole
// strips of 62 lanes x VEC cells per row, the work a wave does per row), and
// deal the items to workgroups.
int schedule_batch_2d(int n_cu, int dtype, int lm, int max_L, const std::vector<SchedField> &fields,
                      int item_cells, int wg_per_cu, std::vector<BatchItem> &sorted, std::vector<int32_t> &first,
                      std::vector<int32_t> &n_items) {
    const int vec = vec_2d(dtype), ce = 62 * vec;
    const int64_t max_units = std::max<int64_t>(1, std::min<int64_t>(item_cells, kFlush2D) / ce);
    std::vector<BatchItem> items;
    std::vector<int64_t> cost;
    n_items.assign(fields.size(), 0);
    for (size_t f = 0; f < fields.size(); ++f) {
        const int64_t strips = (fields[f].w + ce - 1) / ce, units = strips * fields[f].h;
        const int64_t k = (units + max_units - 1) / max_units;  // items of this field
        for (int64_t j = 0; j < k; ++j) {
            const int64_t u0 = units * j / k, u1 = units * (j + 1) / k;
            items.push_back(BatchItem{fields[f].slot, (int32_t)u0, (int32_t)u1, 0});
            cost.push_back(u1 - u0);
        }
        n_items[f] = (int32_t)k;
    }
    const size_t lds = lds_bytes_batch_2d(lm, max_L) + 6 * 1024;
    const int fit = std::max<int>(1, (int)((160 * 1024) / lds));
    const int64_t G = std::min<int64_t>((int64_t)n_cu * std::min(wg_per_cu, fit), (int64_t)items.size());
    const int grid = (int)std::max<int64_t>(1, G);
    deal_items(items, cost, 8, grid, sorted, first);
    return grid;
}

// Tile shape of a batched volume: tx x ty columns (taken by the workgroup's
// 256 threads in rounds) of tz planes, with (tx+2)(ty+2)(tz+2) <= the LDS
// slots of a tile, chosen to minimise a cost model of the tile pass: per tile,
// rounds x planes column steps (about 150 instructions each), the staged
// slots over 256 threads (about 40 each) and a fixed cost per tile.  A 20^3
// volume becomes one 20 x 20 x 20 tile (the generic kernel's 64 x 4 x 16 tiles
// would take ten, a fifth of their slots in the volume).
static TileShape tile_shape_search(int64_t d, int64_t h, int64_t w) {
    TileShape best{std::min<int>(64, (int)w), 1, 1};
    double best_cost = 1e300;
    const int tx = (int)std::min<int64_t>(64, w);
    for (int ty = 1; ty <= std::min<int64_t>(h, 256); ++ty) {
        const int64_t sxy = (int64_t)(tx + 2) * (ty + 2);
        const int64_t tz_max = kBatch3DTileElems / sxy - 2;
        if (tz_max < 1) break;
        const int tz = (int)std::min<int64_t>({d, tz_max, 64});
        const int64_t tiles = ((w + tx - 1) / tx) * ((h + ty - 1) / ty) * ((d + tz - 1) / tz);
        const int64_t rounds = ((int64_t)tx * ty + 255) / 256;
        const double per_tile = 150.0 * rounds * tz + 40.0 * ((sxy * (tz + 2) + 255) / 256) + 300.0;
        const double cost = (double)tiles * per_tile;
        if (cost < best_cost) {
            best_cost = cost;
            best = TileShape{tx, ty, tz};
        }
    }
    return best;
}

// (memoised per thread: batches repeat the same few shapes thousands of times)
TileShape tile_shape_3d(int64_t d, int64_t h, int64_t w) {
    struct Entry {
        int64_t d, h, w;
        TileShape ts;
    };
    thread_local Entry cache[64] = {};
    thread_local int next = 0;
    for (const Entry &e : cache)
        if (e.d == d && e.h == h && e.w == w) return e.ts;
    const TileShape ts = tile_shape_search(d, h, w);
    cache[next] = Entry{d, h, w, ts};
    next = (next + 1) % 64;
    return ts;
}

// items of whole tiles of one volume (at most kFlush3D voxels and about
// item_cells per item, so that the packed LDS bins cannot overflow); appends
// to items / cost, returns the item count
static int64_t tile_items(int32_t slot, int64_t d, int64_t h, int64_t w, const TileShape &ts, int item_cells,
                          std::vector<BatchItem> &items, std::vector<int64_t> &cost) {
    const int64_t tv = (int64_t)ts.tx * ts.ty * ts.tz;
    const int64_t max_tiles = std::max<int64_t>(1, std::min<int64_t>(item_cells, kFlush3D) / tv);
    const int64_t tiles = ((w + ts.tx - 1) / ts.tx) * ((h + ts.ty - 1) / ts.ty) * ((d + ts.tz - 1) / ts.tz);
    const int64_t tile_cost = (((int64_t)ts.tx * ts.ty + 255) / 256) * ts.tz + 2;
    const int64_t k = (tiles + max_tiles - 1) / max_tiles;
    for (int64_t j = 0; j < k; ++j) {
        const int64_t u0 = tiles * j / k, u1 = tiles * (j + 1) / k;
        items.push_back(BatchItem{slot, (int32_t)u0, (int32_t)u1, 0});
        cost.push_back((u1 - u0) * tile_cost);
    }
    return k;
}

int schedule_batch_3d(int n_cu, int max_L, const std::vector<SchedField> &fields, int item_cells, int wg_per_cu,
                      std::vector<BatchItem> &sorted, std::vector<int32_t> &first, std::vector<int32_t> &n_items) {
    std::vector<BatchItem> items;
    std::vector<int64_t> cost;
    n_items.assign(fields.size(), 0);
    for (size_t f = 0; f < fields.size(); ++f) {
        const TileShape ts = tile_shape_3d(fields[f].d, fields[f].h, fields[f].w);
        n_items[f] = (int32_t)tile_items(fields[f].slot, fields[f].d, fields[f].h, fields[f].w, ts, item_cells, items,
                                         cost);
    }
    const size_t lds = lds_bytes_batch_3d(max_L) + 2 * kBatch3DTileElems + 13 * 1024;  // + tables, scan
    const int fit = std::max<int>(1, (int)((160 * 1024) / lds));
    const int64_t G = std::min<int64_t>((int64_t)n_cu * std::min(wg_per_cu, fit), (int64_t)items.size());
    const int grid = (int)std::max<int64_t>(1, G);
    deal_items(items, cost, 4, grid, sorted, first);
    return grid;
}

int schedule_4d(int n_cu, int L, int64_t n_vol, int64_t d, int64_t h, int64_t w, const TileShape &ts,
                std::vector<BatchItem> &sorted, std::vector<int32_t> &first) {
    std::vector<BatchItem> items;
    std::vector<int64_t> cost;
    for (int64_t v = 0; v < n_vol; ++v) tile_items((int32_t)v, d, h, w, ts, 64 * 1024, items, cost);
    const size_t lds = lds_bytes_4d(L) + 2 * kBatch3DTileElems + 3 * 1024;
    const int fit = std::max<int>(1, (int)((160 * 1024) / lds));
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)n_cu * std::min(4, fit),
                                                                 (int64_t)items.size()));
    deal_items(items, cost, 4, grid, sorted, first);
    return grid;
}

}  // namespace ecc
