// Tile-shape table.  Defaults come from measurements on MI355X; the tuner
// replaces entries through pl_tune_set.
#include "tuning.h"
#include "tiles.h"

#include <atomic>
#include <mutex>

namespace pl {

namespace {

std::mutex g_mu;
TileCfg g_cfg[kNumStages][kMaxRadius + 1] = {
    // Laplacian: {th, tw, fuse} per radius (3x3, 5x5: the fused path's
    // measured best on a 480x640 and a 128x2048 frame)
    {{0, 0, 0}, {16, 16, 4}, {16, 16, 2}, {8, 32, 1}, {8, 32, 1}},
    // bilateral
    {{0, 0, 0}, {8, 32, 1}, {2, 32, 1}, {8, 32, 1}, {8, 32, 1}},
    // batched Laplacian (a 64-frame mix)
    {{0, 0, 0}, {16, 16, 4}, {16, 16, 2}, {8, 32, 1}, {8, 32, 1}},
    // batched bilateral
    {{0, 0, 0}, {8, 32, 1}, {16, 16, 1}, {8, 32, 1}, {8, 32, 1}},
    // Laplacian, small frames (120x160, 64x1024)
    {{0, 0, 0}, {8, 16, 4}, {8, 16, 2}, {8, 32, 1}, {8, 32, 1}},
    // bilateral, small frames
    {{0, 0, 0}, {4, 32, 2}, {2, 32, 1}, {4, 16, 1}, {4, 16, 1}},
};

// gfx950 LDS per workgroup, less room for the batched kernels' static LDS
constexpr size_t kLdsMax = 156 * 1024;

}  // namespace

size_t cfg_lds_bytes(Stage s, int R, TileCfg c) {
    return is_laplacian(s) ? lap_lds_bytes(R, c.fuse, c.th, c.tw)
                           : bil_lds_bytes(R, c.fuse, c.th, c.tw, bil_waves(R, s == kStageBatchBilateral));
}

TileCfg tile_cfg(Stage s, int R) {
    std::lock_guard<std::mutex> g(g_mu);
    return g_cfg[s][R];
}

bool set_tile_cfg(Stage s, int R, TileCfg c) {
    if (R < 1 || R > kMaxRadius || c.th < 1 || c.tw < 1 || c.fuse < 1 || c.fuse > 8) return false;
    if (c.th * c.tw > 64 * kTileBlock) return false;
    if (cfg_lds_bytes(s, R, c) > kLdsMax) return false;
    std::lock_guard<std::mutex> g(g_mu);
    g_cfg[s][R] = c;
    return true;
}

pl_status allow_lds(const void *kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return PL_OK;
    return hip_check(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)bytes),
                     "hipFuncSetAttribute");
}

}  // namespace pl
