// Host-side launch planning (kgs_stream3d_plan.cpp, kgs_launch.cpp).
#pragma once

namespace kgs {

// Compute units of the current device (256, that of MI355X, when no device
// is visible), cached per device.
int device_cus();

// Estimated duration, in plane-steps, of a four-sweep z-streaming launch
// over grids n[0..count) with the tile_x x tile_y tile and plane chunk
// `chunk` on a device of `cus` compute units (one workgroup per CU).
double stream3d_launch_steps(const int *n, int count, int tile_x, int tile_y, int chunk, int cus);

// The plane chunk (8..128) whose launch is estimated to end first, the
// longer of two within 1%.  stream3d_list_chunk: the same for a
// member-list launch of that precision on the current device.
int stream3d_chunk(const int *n, int count, int tile_x, int tile_y, int cus);
int stream3d_list_chunk(const int *n, int count, int elem_bytes);

}  // namespace kgs
