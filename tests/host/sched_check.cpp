// Host checks of the work schedules and of the contribution tables, built
// with AddressSanitizer and UndefinedBehaviorSanitizer (test_host_sanitizers.py).
//
// Every schedule must cover each field's units (2D strips x rows, 3D tiles)
// exactly once, keep every item within the cells the packed LDS bins may see
// between drains, group the items by workgroup consistently, and keep every
// tile's staged levels within the LDS slots of a tile: a schedule that broke
// one of these would make the kernels read or write out of bounds.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "ecc_schedule.h"

namespace ecc {
// the library's error recorder lives in its runtime, which is not linked here
ecc_status fail(ecc_status s, const std::string &) { return s; }
}  // namespace ecc

using namespace ecc;

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);    \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

// items grouped by workgroup; per field (slot), its items cover [0, units) once
static void check_schedule(const std::vector<BatchItem> &sorted, const std::vector<int32_t> &first, int grid,
                           const std::vector<int64_t> &units, const std::vector<int32_t> *n_items,
                           int64_t max_units_per_item) {
    CHECK(grid >= 1);
    CHECK((int)first.size() == grid + 1);
    CHECK(first[0] == 0 && first[grid] == (int32_t)sorted.size());
    for (int g = 0; g < grid; ++g) CHECK(first[g] <= first[g + 1]);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per(units.size());
    for (const BatchItem &it : sorted) {
        CHECK(it.field >= 0 && it.field < (int32_t)units.size());
        CHECK(it.u0 >= 0 && it.u0 < it.u1 && it.u1 <= units[it.field]);
        CHECK(it.u1 - it.u0 <= max_units_per_item);
        per[it.field].push_back({it.u0, it.u1});
    }
    for (size_t f = 0; f < units.size(); ++f) {
        auto &v = per[f];
        std::sort(v.begin(), v.end());
        int64_t at = 0;
        for (auto &r : v) {
            CHECK(r.first == at);
            at = r.second;
        }
        CHECK(at == units[f]);
        if (n_items) CHECK((*n_items)[f] == (int32_t)v.size());
    }
}

int main(int argc, char **argv) {
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 200;
    std::mt19937_64 rng(12345);
    auto uni = [&](int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); };
    for (int r = 0; r < rounds; ++r) {
        // 2D batches
        {
            const int dtype = (int)uni(1, 3), lm = dtype == 3 ? (int)uni(2, 3) : (int)uni(0, 1);
            const int n = (int)uni(1, 60), max_L = (int)uni(1, kBatchMaxLevels);
            std::vector<SchedField> f;
            std::vector<int64_t> units;
            const int ce = 62 * vec_2d(dtype);
            for (int i = 0; i < n; ++i) {
                const int64_t h = uni(1, r % 7 == 0 ? 20000 : 2000), w = uni(1, r % 5 == 0 ? 40000 : 3000);
                f.push_back(SchedField{i, h, w});
                units.push_back(((w + ce - 1) / ce) * h);
            }
            std::vector<BatchItem> sorted;
            std::vector<int32_t> first, n_items;
            const int item_cells = (int)uni(1024, 1 << 20);
            const int grid = schedule_batch_2d(256, dtype, lm, max_L, f, item_cells, (int)uni(1, 8), sorted, first,
                                               n_items);
            const int64_t max_units = std::max<int64_t>(1, std::min<int64_t>(item_cells, kFlush2D) / ce);
            check_schedule(sorted, first, grid, units, &n_items, max_units);
            CHECK(max_units * ce <= kFlush2D || max_units == 1);
        }
        // 3D batches and their tile shapes
        {
            const int n = (int)uni(1, 40);
            std::vector<SchedField> f;
            std::vector<int64_t> units;
            int64_t max_tv = 1;
            for (int i = 0; i < n; ++i) {
                const int64_t d = uni(1, 200), h = uni(1, 300), w = uni(1, 300);
                f.push_back(SchedField{i, h, w, d});
                const TileShape ts = tile_shape_3d(d, h, w);
                CHECK(ts.tx >= 1 && ts.ty >= 1 && ts.tz >= 1 && ts.tx <= 64);
                CHECK((int64_t)(ts.tx + 2) * (ts.ty + 2) * (ts.tz + 2) <= kBatch3DTileElems);
                CHECK(ts.tx <= w && ts.ty <= h && ts.tz <= d);
                units.push_back(((w + ts.tx - 1) / ts.tx) * ((h + ts.ty - 1) / ts.ty) * ((d + ts.tz - 1) / ts.tz));
                max_tv = std::max<int64_t>(max_tv, (int64_t)ts.tx * ts.ty * ts.tz);
                const TileShape again = tile_shape_3d(d, h, w);  // memoised: the same answer
                CHECK(again.tx == ts.tx && again.ty == ts.ty && again.tz == ts.tz);
            }
            std::vector<BatchItem> sorted;
            std::vector<int32_t> first, n_items;
            const int grid = schedule_batch_3d(256, (int)uni(1, kBatchMaxLevels), f, (int)uni(1024, 1 << 20),
                                               (int)uni(1, 8), sorted, first, n_items);
            check_schedule(sorted, first, grid, units, &n_items, INT32_MAX);
            for (const BatchItem &it : sorted) {  // voxels an item adds to one workgroup's bins
                const TileShape ts = tile_shape_3d(f[it.field].d, f[it.field].h, f[it.field].w);
                CHECK((int64_t)(it.u1 - it.u0) * ts.tx * ts.ty * ts.tz <= std::max<int64_t>(kFlush3D, max_tv));
            }
        }
        // 4D
        {
            const int64_t a = uni(1, 30), d = uni(1, 60), h = uni(1, 60), w = uni(1, 60);
            const int64_t n_vol = 2 * a + 1;
            const TileShape ts = tile_shape_3d(d, h, w);
            std::vector<BatchItem> sorted;
            std::vector<int32_t> first;
            const int grid = schedule_4d(256, (int)uni(1, kBatchMaxLevels), n_vol, d, h, w, ts, sorted, first);
            const int64_t tiles = ((w + ts.tx - 1) / ts.tx) * ((h + ts.ty - 1) / ts.ty) * ((d + ts.tz - 1) / ts.tz);
            check_schedule(sorted, first, grid, std::vector<int64_t>(n_vol, tiles), nullptr, INT32_MAX);
        }
    }
    // contribution tables: every entry computed, within its documented range
    for (int conn : {8, 4}) {
        int32_t t[16][4];
        vertex_table_2d(conn, t);
        for (int k = 0; k < 4; ++k) CHECK(t[0][k] == 0);  // an empty quadrant contributes nothing
        int32_t delta[256][3];
        cell_delta_table_2d(conn, delta);
        for (int p = 0; p < 256; ++p) {
            CHECK(delta[p][0] >= -3 && delta[p][0] <= 1);  // EC change of a pixel entering
            CHECK(delta[p][1] >= -4 && delta[p][1] <= 4);  // perimeter change
            CHECK(delta[p][2] == 1);                       // area change
        }
    }
    for (int conn : {26, 6}) {
        int32_t t[256][4];
        vertex_table_3d(conn, t);
        for (int k = 0; k < 4; ++k) CHECK(t[0][k] == 0);
    }
    int32_t crease[256], cls[256][5];
    crease_delta_table_2d(crease);
    class_delta_table_2d(cls);
    for (int m = 0; m < 16; ++m) CHECK(vertex_class_2d(m) >= -1 && vertex_class_2d(m) < 5);
    for (int m = 0; m < 256; ++m) CHECK(octant_class_3d(m) >= -1 && octant_class_3d(m) < 21);
    std::printf("schedules and tables: %d rounds OK\n", rounds);
    return 0;
}
