// Host-side launch planning (kgs_plan.cpp, kgs_launch.cpp).
#pragma once

#include <cstdint>

namespace kgs {

// Compute units of the current device (256, that of MI355X, when no device
// is visible), cached per device.
int device_cus();

// Planes per chunk of an n-plane grid in a launch of nominal plane chunk
// `chunk`: the equal split into as many chunks, ceil(n / ceil(n / chunk)),
// so that no chunk of a grid is much shorter than its others.
int member_chunk(int n, int chunk);

// Estimated duration, in plane-steps, of a four-sweep z-streaming launch
// over grids n[0..count) with the tile_x x tile_y tile and nominal plane
// chunk `chunk` (member_chunk for each grid) on a device of `cus` compute
// units (one workgroup per CU).
double stream3d_launch_steps(const int *n, int count, int tile_x, int tile_y, int chunk, int cus);

// The nominal plane chunk (8..128) whose launch is estimated to end
// first, the longer of two within 1%, from 128, 96, 64, 48, 32, 24, 16, 12
// and 8 planes and, for a single grid (count 1), its equal splits
// ceil(n / k); for a single grid the result is its member_chunk.
int stream3d_chunk(const int *n, int count, int tile_x, int tile_y, int cus);

// Tile and plane chunk of a four-sweep z-streaming launch over one n^3 grid
// with state elements of elem_bytes.  float32: 16x32 tiles from n = 128,
// else 16x16.  float64: 32x13 (12 waves) when its launch is estimated to
// end at least 2% before that of 16x16 (8 waves), the plane-steps of a
// 32x13 workgroup counted 1.45 times those of a 16x16 one; else 16x16.
void stream3d_plan(int n, int elem_bytes, int cus, int *tile_x, int *tile_y, int *chunk);

// The same for a member-list launch over grids n[0..count) of one
// precision on the current device: float32 takes its default list tile
// (stream3d_list_tile), float64 the rule above over the whole list.
void stream3d_list_plan(const int *n, int count, int elem_bytes, int *tile_x, int *tile_y,
                        int *chunk);

// Grid of the streaming energy reduction of a 2-D or 3-D grid (workgroups
// of 256 columns of a plane of axis 0, bx per plane, by chunks of `chunk`
// planes): the closing form holds three workgroups per CU, so the chunk is
// the one that minimises whole rounds of 3 * cus workgroups times planes
// per workgroup (plus 2 for its first loads).  False for 1-D grids and
// planes of more than 2048 * 256 columns, which do not stream.
bool energy_grid(int dim, int n, int cus, int64_t *bx, int64_t *by, int64_t *chunk);

}  // namespace kgs
