// Prints the launch estimate and the chosen chunk of the z-streaming launch
// planner for one group of grids: plan_driver tile_x tile_y cus chunk n...
// (chunk 0: only the chosen chunk); or the energy reduction's grid:
// plan_driver energy dim n cus; or a single grid's tile and chunk:
// plan_driver plan n elem_bytes cus.  The planner's two device-facing
// helpers are stood in for here: no GPU is needed.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "kgs_plan.h"

namespace kgs {
void stream3d_list_tile(int elem_bytes, int *tile_x, int *tile_y)
{
    *tile_x = 16;
    *tile_y = elem_bytes == 8 ? 16 : 32;
}
int device_cus() { return 256; }
}  // namespace kgs

int main(int argc, char **argv)
{
    if (argc == 5 && std::string(argv[1]) == "energy") {
        // plan_driver energy dim n cus: bx by chunk (0 0 0: no streaming grid)
        int64_t bx = 0, by = 0, chunk = 0;
        const bool ok = kgs::energy_grid(std::atoi(argv[2]), std::atoi(argv[3]),
                                         std::atoi(argv[4]), &bx, &by, &chunk);
        std::printf("%lld %lld %lld\n", static_cast<long long>(ok ? bx : 0),
                    static_cast<long long>(ok ? by : 0), static_cast<long long>(ok ? chunk : 0));
        return 0;
    }
    if (argc == 5 && std::string(argv[1]) == "plan") {
        // plan_driver plan n elem_bytes cus: tile_x tile_y chunk
        int tx = 0, ty = 0, chunk = 0;
        kgs::stream3d_plan(std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), &tx, &ty,
                           &chunk);
        std::printf("%d %d %d\n", tx, ty, chunk);
        return 0;
    }
    if (argc < 6) return 2;
    const int tx = std::atoi(argv[1]), ty = std::atoi(argv[2]), cus = std::atoi(argv[3]);
    const int chunk = std::atoi(argv[4]);
    std::vector<int> n;
    for (int i = 5; i < argc; ++i) n.push_back(std::atoi(argv[i]));
    const int count = static_cast<int>(n.size());
    const int best = kgs::stream3d_chunk(n.data(), count, tx, ty, cus);
    const double est = chunk > 0 ? kgs::stream3d_launch_steps(n.data(), count, tx, ty, chunk, cus) : 0.0;
    int t64[3], t32[3];
    kgs::stream3d_list_plan(n.data(), count, 8, &t64[0], &t64[1], &t64[2]);
    kgs::stream3d_list_plan(n.data(), count, 4, &t32[0], &t32[1], &t32[2]);
    std::printf("%d %.6f %d %d %d %d %d %d\n", best, est, t64[0], t64[1], t64[2], t32[0], t32[1],
                t32[2]);
    return 0;
}
