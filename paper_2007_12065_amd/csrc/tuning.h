// Runtime tile shapes and sweep fusion, read by every launcher and set by the
// tuner (pl_tune_set).  The only mutable global state of the library.
#pragma once

#include "common.h"

namespace pl {

enum Stage {
    kStageLaplacian = 0,
    kStageBilateral = 1,
    kStageBatchLaplacian = 2,      // the batched path's entries
    kStageBatchBilateral = 3,
    kStageLaplacianSmall = 4,      // single frames of at most kSmallFramePoints points
    kStageBilateralSmall = 5,
    kNumStages = 6
};
inline bool is_laplacian(Stage s) {
    return s == kStageLaplacian || s == kStageBatchLaplacian || s == kStageLaplacianSmall;
}
// Single frames up to this many points read the *Small entries: a 64 x 1024
// frame has a quarter of the tiles of a 480 x 640 one, and the shapes that
// fill the chip differ.
constexpr long kSmallFramePoints = 1L << 17;
inline Stage frame_stage(bool laplacian, int M, int N) {
    const bool small = (long)M * N <= kSmallFramePoints;
    if (laplacian) return small ? kStageLaplacianSmall : kStageLaplacian;
    return small ? kStageBilateralSmall : kStageBilateral;
}
constexpr int kMaxRadius = 4;                 // kernel sizes 3, 5, 7, 9

struct TileCfg {
    int th, tw;      // tile rows x columns (points for the Laplacian, quads for the bilateral)
    int fuse;        // sweeps fused per launch
};

// Current configuration for a stage and window radius (1..4).
TileCfg tile_cfg(Stage s, int R);
// Replace it; returns false if the shape does not fit the kernels' limits.
bool set_tile_cfg(Stage s, int R, TileCfg c);
// LDS bytes a configuration needs.
size_t cfg_lds_bytes(Stage s, int R, TileCfg c);
// Raise a kernel's dynamic-LDS limit when a configuration needs more than
// the default 64 KB (once per kernel and size).
pl_status allow_lds(const void *kernel, size_t bytes);

}  // namespace pl
