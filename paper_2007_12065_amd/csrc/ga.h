// Gaussian accumulator (Sec. 6.1): internal interface between the C ABI and
// ga.hip.
#pragma once

#include "common.h"

namespace pl {

constexpr int kGaMaxLevel = 5;           // 20480 cells: counts fit the LDS histogram
constexpr int kGaMaxCells = 32768;       // caller-given cells (16-bit cell ids, LDS)

size_t ga_level_workspace(int level);
size_t ga_cells_workspace(const float *cells, int n_cells);
pl_status ga_create_level(int level, void *ws, hipStream_t s, pl_ga_s **out);
pl_status ga_create_cells(const float *cells, int n_cells, void *ws, hipStream_t s,
                          pl_ga_s **out);
size_t ga_bytes(const pl_ga_s *g);
int ga_cell_count(const pl_ga_s *g);
const float *ga_cells(const pl_ga_s *g);
pl_status ga_integrate(const pl_ga_s *g, const void *normals, pl_dtype ndt,
                       const int32_t *n_dev, int cap, int stride, uint32_t *counts,
                       int32_t *cell_out, hipStream_t s);
void ga_destroy(pl_ga_s *g);

}  // namespace pl
