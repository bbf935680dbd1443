// Autotuner: times candidate launch configurations of a simulation on a copy
// of its current state and keeps the fastest.  Every configuration computes
// bitwise the same state (same-colour points are independent), so tuning
// only changes speed; the state is restored after every candidate.  Winners
// are cached per (dimension, n, precision, GPU architecture) for the
// process and, when the environment variable KGS_TUNE_CACHE names a file,
// in that file: one line per winner, appended, read back by later calls in
// any process (the last line for a key wins).
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "kgs.h"
#include "kgs_trace.h"
#include "kgs_internal.h"
#include "kgs_sim.h"

namespace {

using Key = std::tuple<int, int, int, std::string>;  // dim, n, precision, architecture
std::map<Key, kgs_tuning> g_cache;
std::mutex g_cache_mutex;
std::string g_loaded_file;  // the cache file whose lines are in g_cache

constexpr const char *kFileTag = "kgs-tune-v1";

// Architecture name of a device (e.g. gfx950:sramecc+:xnack-), or "" on a
// runtime error.
std::string arch_of(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return std::string();
    std::string a(prop.gcnArchName);
    for (char &ch : a)
        if (ch == ' ') ch = '_';
    return a;
}

std::string cache_file()
{
    const char *p = std::getenv("KGS_TUNE_CACHE");
    return p ? std::string(p) : std::string();
}

// Reads the cache file's lines into g_cache once per file name (caller
// holds g_cache_mutex).  Lines that do not parse are skipped.
void load_file_locked(const std::string &path)
{
    if (path.empty() || path == g_loaded_file) return;
    g_loaded_file = path;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char tag[32], arch[256];
        int dim, n, prec;
        kgs_tuning t;
        std::memset(&t, 0, sizeof(t));
        if (std::sscanf(line, "%31s %255s %d %d %d %d %d %d %d %d %d", tag, arch, &dim, &n, &prec,
                        &t.kernel, &t.block, &t.tile_x, &t.tile_y, &t.chunk,
                        &t.steps_per_launch) == 11 &&
            std::strcmp(tag, kFileTag) == 0)
            g_cache[Key{dim, n, prec, std::string(arch)}] = t;
    }
    std::fclose(f);
}

// Appends a winner to the cache file (caller holds g_cache_mutex).
void append_file_locked(const std::string &path, const Key &k, const kgs_tuning &t)
{
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %s %d %d %d %d %d %d %d %d %d\n", kFileTag, std::get<3>(k).c_str(),
                 std::get<0>(k), std::get<1>(k), std::get<2>(k), t.kernel, t.block, t.tile_x,
                 t.tile_y, t.chunk, t.steps_per_launch);
    std::fclose(f);
}

std::vector<kgs_tuning> candidates(const kgs_sim *s)
{
    // the library's own choice first, so that tuning never loses to it
    std::vector<kgs_tuning> out{kgs::default_tuning_of(s->cfg)};
    auto sweep = [&](int block) {
        kgs_tuning t;
        std::memset(&t, 0, sizeof(t));
        t.kernel = KGS_KERNEL_SWEEP;
        t.block = block;
        out.push_back(t);
    };
    for (int b : {128, 256, 512}) sweep(b);
    if (s->cfg.dim == 2) {
        for (int chunk : {8, 16, 32, 64, 128})
            for (int spl : {1, 2}) {
                if (kgs::stream2d_tasks(s->geo.n, chunk) < 1) continue;
                kgs_tuning t;
                std::memset(&t, 0, sizeof(t));
                t.kernel = KGS_KERNEL_STREAM;
                t.block = 256;
                t.chunk = chunk;
                t.steps_per_launch = spl;
                out.push_back(t);
            }
        const int eb = s->cfg.precision == KGS_FP32 ? 4 : 8;
        const int tiles[][3] = {{8, 8, 2},   {8, 16, 2},  {16, 16, 2}, {16, 32, 2},
                                {32, 16, 2}, {32, 32, 2}, {16, 16, 1}, {32, 32, 1},
                                {16, 16, 4}, {16, 32, 4}, {32, 32, 4}};
        for (const auto &tl : tiles) {
            if (!kgs::tile2d_shape_ok(s->geo, tl[0], tl[1], 2 * tl[2], eb)) continue;
            kgs_tuning t;
            std::memset(&t, 0, sizeof(t));
            t.kernel = KGS_KERNEL_TILE;
            t.block = 256;
            t.tile_y = tl[0];
            t.tile_x = tl[1];
            t.steps_per_launch = tl[2];
            out.push_back(t);
        }
    }
    if (s->cfg.dim == 3) {
        const int eb = s->cfg.precision == KGS_FP32 ? 4 : 8;
        const int shapes[][4] = {
            {16, 16, 128, 2}, {16, 17, 64, 2}, {16, 16, 64, 2}, {12, 24, 128, 2}, {8, 32, 128, 2},
            {32, 16, 64, 2},  {32, 16, 128, 2}, {16, 40, 64, 2}, {32, 16, 64, 1}, {64, 8, 64, 1},
            {16, 32, 64, 1},  {32, 8, 32, 1},   {16, 16, 32, 2}, {32, 20, 64, 2},
            {16, 16, 16, 2},  {16, 16, 8, 2},   {16, 16, 16, 1},  {16, 32, 128, 2},
            {16, 32, 64, 2},  {16, 32, 32, 2},  {16, 32, 16, 2},  {16, 32, 8, 2},
            {32, 13, 128, 2}, {32, 13, 96, 2},  {32, 13, 64, 2},  {32, 13, 48, 2},
        };
        for (const auto &sh : shapes) {
            kgs::StreamShape ss = {sh[0], sh[1], sh[2], sh[3]};
            if (!kgs::stream3d_shape_ok(s->geo, ss, eb)) continue;
            kgs_tuning t;
            std::memset(&t, 0, sizeof(t));
            t.kernel = KGS_KERNEL_STREAM;
            t.block = 256;
            t.tile_x = sh[0];
            t.tile_y = sh[1];
            t.chunk = sh[2];
            t.steps_per_launch = sh[3];
            out.push_back(t);
        }
    }
    return out;
}

// Winners of batch groups (kgs_batch_autotune), keyed by group signature.
std::map<std::string, kgs::GroupTuning> g_groups;
std::string g_groups_loaded;  // the cache file whose group lines are in g_groups
constexpr const char *kGroupTag = "kgs-group-v1";

// Group lines: tag, then the signature's words (architecture, dim,
// precision, member sizes joined by commas), then mode chunk ty tx.
void load_groups_locked(const std::string &path)
{
    if (path.empty() || path == g_groups_loaded) return;
    g_groups_loaded = path;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[8192];
    while (std::fgets(line, sizeof(line), f)) {
        char tag[32], arch[256], sizes[7680];
        int dim, prec;
        kgs::GroupTuning t;
        if (std::sscanf(line, "%31s %255s %d %d %7679s %d %d %d %d", tag, arch, &dim, &prec, sizes,
                        &t.mode, &t.chunk, &t.ty, &t.tx) == 9 &&
            std::strcmp(tag, kGroupTag) == 0)
            g_groups[std::string(arch) + " " + std::to_string(dim) + " " + std::to_string(prec) +
                     " " + sizes] = t;
    }
    std::fclose(f);
}

}  // namespace

namespace kgs {

std::string group_signature(int device, int dim, int precision, std::vector<int> sizes)
{
    std::sort(sizes.begin(), sizes.end());
    std::string s = arch_of(device) + " " + std::to_string(dim) + " " + std::to_string(precision) + " ";
    for (size_t i = 0; i < sizes.size(); ++i) s += (i ? "," : "") + std::to_string(sizes[i]);
    return s;
}

bool group_cache_get(const std::string &sig, GroupTuning &t)
{
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    load_groups_locked(cache_file());
    auto it = g_groups.find(sig);
    if (it == g_groups.end()) return false;
    t = it->second;
    return true;
}

void group_cache_put(const std::string &sig, const GroupTuning &t)
{
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    g_groups[sig] = t;
    const std::string path = cache_file();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %s %d %d %d %d\n", kGroupTag, sig.c_str(), t.mode, t.chunk, t.ty, t.tx);
    std::fclose(f);
}

}  // namespace kgs

extern "C" int kgs_autotune(kgs_sim *s, int32_t steps, int32_t use_cache, kgs_tuning *best)
{
    KGS_TRACE("kgs_autotune");
    if (!s || steps < 1) return KGS_EINVAL;
    const Key key{s->cfg.dim, s->cfg.n, s->cfg.precision, arch_of(s->device)};
    const std::string file = cache_file();
    if (use_cache) {
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        load_file_locked(file);
        auto it = g_cache.find(key);
        // an entry that no longer fits the grid is tuned again
        if (it != g_cache.end() && kgs_set_tuning(s, &it->second) == KGS_OK) {
            if (best) *best = it->second;
            return KGS_OK;
        }
        s->err.clear();
    }
    if (hipSetDevice(s->device) != hipSuccess) return KGS_EDEVICE;
    const size_t bytes = 8 * s->plane_bytes;
    void *backup = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = KGS_OK;
    if (hipMalloc(&backup, bytes) != hipSuccess) {
        s->err = "autotune: no device memory for the state copy";
        return KGS_ENOMEM;
    }
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = KGS_EDEVICE;
    // the state is saved closed and restored closed after every candidate
    if (rc == KGS_OK && kgs::sim_close(s, s->stream) != KGS_OK) rc = KGS_EDEVICE;
    if (rc == KGS_OK &&
        hipMemcpyAsync(backup, s->state, bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        rc = KGS_EDEVICE;
    const kgs_tuning original = s->tuning;
    kgs_tuning winner = original;
    float best_ms = -1.0f;
    if (rc == KGS_OK) {
        for (const kgs_tuning &t : candidates(s)) {
            if (kgs_set_tuning(s, &t) != KGS_OK) continue;
            // a warm-up step, then the faster of two timed calls of `steps`
            // steps (one short sample alone picked configurations that lose
            // in longer runs); the state is restored after the candidate
            if (kgs_step(s, 1) != KGS_OK) break;
            float ms = -1.0f;
            for (int rep = 0; rep < 2 && rc == KGS_OK; ++rep) {
                float m = 0.0f;
                if (hipEventRecord(a, s->stream) != hipSuccess || kgs_step(s, steps) != KGS_OK ||
                    hipEventRecord(b, s->stream) != hipSuccess ||
                    hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&m, a, b) != hipSuccess)
                    rc = KGS_EDEVICE;
                else if (ms < 0.0f || m < ms)
                    ms = m;
            }
            if (rc != KGS_OK) break;
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                winner = t;
            }
            if (hipMemcpyAsync(s->state, backup, bytes, hipMemcpyDeviceToDevice, s->stream) !=
                hipSuccess) {
                rc = KGS_EDEVICE;
                break;
            }
            s->open = false;
        }
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess && rc == KGS_OK) rc = KGS_EDEVICE;
    kgs::FirstError rel;
    if (a) rel(hipEventDestroy(a));
    if (b) rel(hipEventDestroy(b));
    rel(hipFree(backup));
    if (!rel.ok() && rc == KGS_OK) rc = KGS_EDEVICE;
    if (rc != KGS_OK) {
        s->err = "autotune: a HIP call failed";
        kgs_set_tuning(s, &original);
        return rc;
    }
    rc = kgs_set_tuning(s, &winner);
    if (rc == KGS_OK) {
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        g_cache[key] = winner;
        append_file_locked(file, key, winner);
    }
    if (best) *best = winner;
    return rc;
}
