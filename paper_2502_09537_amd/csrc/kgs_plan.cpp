// Launch planning: the plane chunk of z-streaming launches (kgs_stream3d.hip)
// and the grid of the streaming energy reduction (kgs_energy.hip), each the
// one estimated to end first.
#include <algorithm>
#include <cstdint>
#include <functional>
#include <iterator>
#include <queue>
#include <vector>

#include "kgs_internal.h"
#include "kgs_plan.h"

namespace kgs {

// A launch's workgroups are dealt to the 8 XCDs in turn, and xcd_item
// gives XCD x the x-th of 8 contiguous slices of ceil(items / 8) items (the
// last slices shorter); each XCD starts its next item on the first of its
// CUs that is free.  An item of L planes
// takes L + kItemSteps pipeline steps: on MI355X at 256^3 float64 a launch
// of one round of 128-plane items took 260 us, of two rounds of 64-plane
// items 291 us (145.5 per item), which puts the fixed cost of an item
// (pipeline fill and drain, set-up) at 17 plane-steps.
int member_chunk(int n, int chunk)
{
    if (n < 1 || chunk < 1) return chunk;
    const int k = (n + chunk - 1) / chunk;
    return (n + k - 1) / k;
}

double stream3d_launch_steps(const int *n, int count, int tile_x, int tile_y, int chunk, int cus)
{
    constexpr int kItemSteps = 17;
    constexpr int kXcds = 8;
    constexpr int64_t kDealLimit = 16384;  // beyond: 64+ rounds, tail < 2%
    if (count < 1 || cus < 1 || chunk < 1) return 0.0;
    int64_t items = 0;
    double work = 0.0;
    int longest = 0;
    for (int m = 0; m < count; ++m) {
        const int64_t tiles =
            static_cast<int64_t>((n[m] / 2 + tile_x - 1) / tile_x) * ((n[m] + tile_y - 1) / tile_y);
        const int cm = member_chunk(n[m], chunk);
        const int nc = (n[m] + cm - 1) / cm;
        items += tiles * nc;
        work += static_cast<double>(tiles) * (n[m] + static_cast<double>(nc) * kItemSteps);
        longest = std::max(longest, std::min(cm, n[m]) + kItemSteps);
    }
    if (items > kDealLimit) return work / cus + longest;
    // item lengths in item order: per member its tiles first, then its chunks
    std::vector<int> len;
    len.reserve(static_cast<size_t>(items));
    for (int m = 0; m < count; ++m) {
        const int64_t tiles =
            static_cast<int64_t>((n[m] / 2 + tile_x - 1) / tile_x) * ((n[m] + tile_y - 1) / tile_y);
        const int cm = member_chunk(n[m], chunk);
        for (int z0 = 0; z0 < n[m]; z0 += cm)
            len.insert(len.end(), static_cast<size_t>(tiles), std::min(cm, n[m] - z0) + kItemSteps);
    }
    const int groups = cus % kXcds == 0 ? kXcds : 1;
    const int per = cus / groups;
    const int64_t q = (items + groups - 1) / groups;  // items per slice
    double end = 0.0;
    for (int x = 0; x < groups; ++x) {
        std::priority_queue<int64_t, std::vector<int64_t>, std::greater<int64_t>> free_at;
        for (int c = 0; c < per; ++c) free_at.push(0);
        const int64_t first = x * q, last = std::min(items, (x + 1) * q);
        for (int64_t i = first; i < last; ++i) {
            const int64_t t = free_at.top() + len[static_cast<size_t>(i)];
            free_at.pop();
            free_at.push(t);
            end = std::max(end, static_cast<double>(t));
        }
    }
    return end;
}

int stream3d_chunk(const int *n, int count, int tile_x, int tile_y, int cus)
{
    static const int kChunks[] = {128, 96, 64, 48, 32, 24, 16, 12, 8};
    std::vector<int> cands(std::begin(kChunks), std::end(kChunks));
    if (count == 1) {
        // a single grid also tries its equal splits, ceil(n / k) planes
        for (int k = 1; k <= n[0]; ++k) {
            const int c = (n[0] + k - 1) / k;
            if (c < 8) break;
            if (c <= 128) cands.push_back(c);
        }
        std::sort(cands.begin(), cands.end(), std::greater<int>());
        cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
    }
    int best = cands[0];
    double best_t = stream3d_launch_steps(n, count, tile_x, tile_y, best, cus);
    for (int c : cands) {
        const double t = stream3d_launch_steps(n, count, tile_x, tile_y, c, cus);
        if (t < 0.99 * best_t) {
            best = c;
            best_t = t;
        }
    }
    return count == 1 ? member_chunk(n[0], best) : best;
}

// The float64 pipeline holds 162 VGPRs per thread at run-time tile shapes,
// so 12 waves per CU (3 per SIMD) fit.  32x13 is the 12-wave tile whose
// rows are a power of two wide (compressed positions: whole tiles along x
// at power-of-two n); its halo rings add 0.82 of the tile's columns
// against 0.88 for 16x16.  Measured on MI355X, float64, us per 2-step
// launch, 16x16 against 32x13 (each with its planned chunk): 168^3 122 /
// 100-104, 200^3 194 / 170-173, 256^3 236.7 / 238-240, 320^3 620 / 611,
// 334^3 859-863 / 774-784, 352^3 787 / 751, 384^3 943 / 845, 448^3 1547 /
// 1504, 512^3 2020 / 1905, 640^3 4759-4936 / 4093-4372, 734^3 7547-8884 /
// 7518-7525.  Divided by the estimated plane-steps, a 32x13 plane-step
// took 1.36-1.53 times a 16x16 one.  The rule keeps 16x16 at 256^3; with
// equal-split chunks it takes 32x13 at 320^3 (80 planes: 545-555 us
// against 626 for 16x16 with 64) and 734^3 (105 planes: 6470-6493 against
// 7750-7812 for 16x16 with 128).
namespace {

void plan_fp64(const int *n, int count, int cus, int *tile_x, int *tile_y, int *chunk)
{
    constexpr double kWideCost = 1.45, kMargin = 0.98;
    const int c16 = stream3d_chunk(n, count, 16, 16, cus);
    const int cw = stream3d_chunk(n, count, 32, 13, cus);
    const double t16 = stream3d_launch_steps(n, count, 16, 16, c16, cus);
    const double tw = kWideCost * stream3d_launch_steps(n, count, 32, 13, cw, cus);
    const bool wide = tw < kMargin * t16;
    *tile_x = wide ? 32 : 16;
    *tile_y = wide ? 13 : 16;
    *chunk = wide ? cw : c16;
}

}  // namespace

void stream3d_plan(int n, int elem_bytes, int cus, int *tile_x, int *tile_y, int *chunk)
{
    if (elem_bytes == 8) {
        plan_fp64(&n, 1, cus, tile_x, tile_y, chunk);
        return;
    }
    *tile_x = 16;
    *tile_y = n >= 128 ? 32 : 16;
    *chunk = stream3d_chunk(&n, 1, *tile_x, *tile_y, cus);
}

bool energy_grid(int dim, int n, int cus, int64_t *bx, int64_t *by, int64_t *chunk)
{
    constexpr int kBlock = 256, kSlots = 2048, kResident = 3, kStartSteps = 2;
    if (dim < 2 || n < 2 || cus < 1) return false;
    const int64_t cols = dim == 3 ? static_cast<int64_t>(n) * (n / 2) : n / 2;
    const int64_t x = (cols + kBlock - 1) / kBlock;
    if (x > kSlots) return false;
    const int64_t round = static_cast<int64_t>(kResident) * cus;
    double best = -1.0;
    for (int64_t b = 1; b <= n && x * b <= kSlots; ++b) {
        const int64_t c = (n + b - 1) / b;
        const int64_t y = (n + c - 1) / c;  // chunks of c planes actually needed
        const double t = static_cast<double>((x * y + round - 1) / round) * (c + kStartSteps);
        if (best < 0.0 || t < best) {
            best = t;
            *bx = x;
            *by = y;
            *chunk = c;
        }
    }
    return best >= 0.0;
}

void stream3d_list_plan(const int *n, int count, int elem_bytes, int *tile_x, int *tile_y,
                        int *chunk)
{
    const int cus = device_cus();
    if (elem_bytes == 8) {
        plan_fp64(n, count, cus, tile_x, tile_y, chunk);
        return;
    }
    stream3d_list_tile(elem_bytes, tile_x, tile_y);
    *chunk = stream3d_chunk(n, count, *tile_x, *tile_y, cus);
}

}  // namespace kgs
