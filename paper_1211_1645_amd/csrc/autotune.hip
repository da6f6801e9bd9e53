// autotune.hip — picks the sweep schedule of a box: the fused tile kernel
// with the fastest (tile, threads) shape for this grid, timed on the box's
// own state, or the simple per-colour schedule where tiling does not apply.
// The trajectory is independent of the choice (counter-keyed random numbers
// and independent same-colour cells), so tuning can never change results.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>
#include <mutex>
#include <tuple>

#include "mpmc_host.hpp"

using namespace mpmc;

namespace {
std::mutex g_mu;
std::map<std::tuple<int, uint32_t, uint32_t>, FusedShape> g_cache;  // (device, M, n_trial)

// The file named by MPMC_TUNE_CACHE, if set, keeps choices across
// processes: one line per choice, "<arch> <CUs> <M> <n_trial> <tile>
// <threads>".  A line is used only if its shape is one the library has and
// fits the box; a tuned choice is appended.
std::string device_id(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    char buf[300];
    std::snprintf(buf, sizeof buf, "%s %d", prop.gcnArchName, prop.multiProcessorCount);
    for (char *c = buf; *c; ++c)
        if (*c == '\n') *c = ' ';
    return std::string(buf);
}

bool file_lookup(const std::string &id, uint32_t M, uint32_t n_trial, const BoxView &v, FusedShape *out) {
    const char *path = std::getenv("MPMC_TUNE_CACHE");
    if (!path || !*path || id.empty()) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512], arch[256];
    bool hit = false;
    uint32_t n = 0;
    const FusedShape *shapes = fused_shapes(&n);
    while (std::fgets(line, sizeof line, f)) {
        int cus = 0;
        unsigned m = 0, nt = 0, tile = 0, threads = 0;
        if (std::sscanf(line, "%255s %d %u %u %u %u", arch, &cus, &m, &nt, &tile, &threads) != 6) continue;
        char want[300];
        std::snprintf(want, sizeof want, "%s %d", arch, cus);
        if (id != want || m != M || nt != n_trial) continue;
        for (uint32_t i = 0; i < n; ++i)
            if (shapes[i].tile == tile && shapes[i].threads == threads && fused_supported(v, shapes[i])) {
                *out = shapes[i];
                hit = true;  // the last valid line wins
            }
    }
    std::fclose(f);
    return hit;
}

void file_store(const std::string &id, uint32_t M, uint32_t n_trial, const FusedShape &s) {
    const char *path = std::getenv("MPMC_TUNE_CACHE");
    if (!path || !*path || id.empty()) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;  // the file is a convenience: tuning stands without it
    std::fprintf(f, "%s %u %u %u %u\n", id.c_str(), M, n_trial, s.tile, s.threads);
    std::fclose(f);
}
}  // namespace

// Times `reps` launches of one shape reading the current buffer and writing
// the other one, with no canonical output.  The canonical state (moved into
// C by the caller first) and the sweep counter are untouched; the trial
// counters are restored afterwards by the caller.
static int time_shape(Box *b, const FusedShape &s, int reps, float *ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(MPMC_EDEVICE, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MPMC_EDEVICE, "hipEventCreate");
    }
    BoxView v = b->view(b->cur);
    v.cnt_can = nullptr;
    v.x_can = v.y_can = nullptr;
    v.tag_can = nullptr;
    for (int r = 0; r < 3; ++r) launch_fused_sweep(v, s, b->stream);
    hipError_t e = hipEventRecord(e0, b->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch_fused_sweep(v, s, b->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(MPMC_EDEVICE, "autotune timing: %s", hipGetErrorString(e));
    *ms = t / reps;
    return MPMC_OK;
}

static int autotune(Box *b, FusedShape *best) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MPMC_EDEVICE, "hipGetDevice");
    const auto key = std::make_tuple(dev, b->g.M, b->p.n_trial);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) { *best = it->second; return MPMC_OK; }
    }
    const std::string id = device_id(dev);
    if (file_lookup(id, b->g.M, b->p.n_trial, b->view(b->cur), best)) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = *best;
        return MPMC_OK;
    }
    int rc = b->materialize();
    if (rc) return rc;
    rc = b->read_scalars();
    if (rc) return rc;
    const DevScalars saved = b->host;
    uint32_t n = 0;
    const FusedShape *shapes = fused_shapes(&n);
    float best_ms = 1e30f;
    bool found = false;
    const BoxView v = b->view(b->cur);
    // three interleaved rounds, best time per shape, so that one noisy
    // measurement does not decide
    std::vector<float> t(n, 1e30f);
    for (int round = 0; round < 3; ++round)
        for (uint32_t i = 0; i < n; ++i) {
            if (!fused_supported(v, shapes[i])) continue;
            float ms;
            rc = time_shape(b, shapes[i], 10, &ms);
            if (rc) return rc;
            t[i] = ms < t[i] ? ms : t[i];
        }
    for (uint32_t i = 0; i < n; ++i)
        if (t[i] < best_ms) { best_ms = t[i]; *best = shapes[i]; found = true; }
    // restore the counters the timing launches advanced
    if (hipMemcpyAsync(b->dev, &saved, sizeof(DevScalars), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return fail(MPMC_EDEVICE, "restoring counters after autotune");
    b->host = saved;
    if (!found) return fail(MPMC_EINVAL, "no fused shape fits this box");
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = *best;
    file_store(id, b->g.M, b->p.n_trial, *best);
    return MPMC_OK;
}

static uint32_t default_threads(uint32_t tile) {
    return tile <= 8 ? 64 : tile <= 34 ? 256 : tile <= 48 ? 512 : 1024;
}

int Box::choose_schedule() {
    const BoxView v = view(cur);
    FusedShape s{p.tile, default_threads(p.tile)};
    switch (p.schedule) {
    case MPMC_SCHED_SIMPLE:
        sched = MPMC_SCHED_SIMPLE;
        shape = FusedShape{0, 0};
        graph_sweeps = 32;
        return MPMC_OK;
    case MPMC_SCHED_FUSED:
        if (!fused_supported(v, s))
            return fail(MPMC_EINVAL, "tile %u does not fit this box (even, tile + 8 <= M, cap 4)", p.tile);
        sched = MPMC_SCHED_FUSED;
        shape = s;
        graph_sweeps = 128;
        return MPMC_OK;
    default: {  // AUTO
        if (p.tile && fused_supported(v, s)) {
            sched = MPMC_SCHED_FUSED;
            shape = s;
            graph_sweeps = 128;
            return MPMC_OK;
        }
        uint32_t n = 0;
        const FusedShape *shapes = fused_shapes(&n);
        bool any = false;
        for (uint32_t i = 0; i < n; ++i) any = any || fused_supported(v, shapes[i]);
        if (!any || !placed) {
            sched = MPMC_SCHED_SIMPLE;
            shape = FusedShape{0, 0};
            graph_sweeps = 32;
            return MPMC_OK;
        }
        FusedShape best;
        int rc = autotune(this, &best);
        if (rc) return rc;
        sched = MPMC_SCHED_FUSED;
        shape = best;
        graph_sweeps = 128;
        return MPMC_OK;
    }
    }
}

extern "C" int mpmc_set_schedule(mpmc_box bh, uint32_t schedule, uint32_t tile, uint32_t threads) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = reinterpret_cast<Box *>(bh);
    if (schedule == MPMC_SCHED_SIMPLE) {
        b->sched = MPMC_SCHED_SIMPLE;
        b->shape = FusedShape{0, 0};
        b->graph_sweeps = 32;
        return MPMC_OK;
    }
    if (schedule == MPMC_SCHED_FUSED) {
        FusedShape s{tile, threads ? threads : default_threads(tile)};
        if (!fused_supported(b->view(b->cur), s))
            return fail(MPMC_EINVAL, "shape (%u, %u) not available for this box", tile, s.threads);
        b->sched = MPMC_SCHED_FUSED;
        b->shape = s;
        b->graph_sweeps = 128;
        return MPMC_OK;
    }
    if (schedule == MPMC_SCHED_AUTO) {
        const uint32_t keep = b->p.schedule;
        b->p.schedule = MPMC_SCHED_AUTO;
        const uint32_t keep_tile = b->p.tile;
        b->p.tile = 0;
        int rc = b->choose_schedule();
        b->p.schedule = keep;
        b->p.tile = keep_tile;
        return rc;
    }
    return fail(MPMC_EINVAL, "unknown schedule %u", schedule);
}

extern "C" int mpmc_set_graphs(mpmc_box bh, uint32_t sweeps_per_graph) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = reinterpret_cast<Box *>(bh);
    if (sweeps_per_graph != 0 && (sweeps_per_graph & 1u))
        return fail(MPMC_EINVAL, "sweeps per graph must be even (double-buffered state)");
    b->use_graphs = sweeps_per_graph != 0;
    if (sweeps_per_graph) b->graph_sweeps = sweeps_per_graph;
    return MPMC_OK;
}
