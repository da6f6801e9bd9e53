// batch.hip — many independent boxes of uneven N and eta swept together:
// one persistent kernel launch per sweep strides over a work list of
// (box, tile) items, and long runs replay a captured graph of such launches
// with one batched counter update at the end.  Each box keeps its own
// geometry, seed, counters and contact histogram, so box b evolves exactly
// as a single box with the same parameters would.
#include <math.h>
#include <string.h>

#include <vector>

#include "mpmc_host.hpp"

using namespace mpmc;

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MPMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

namespace {
struct Batch {
    std::vector<Box *> boxes;
    mpmc_params p{};
    hipStream_t stream = nullptr, cap_stream = nullptr;
    BoxView *d_views = nullptr;    // per box and buffer parity
    BoxView *d_views_t = nullptr;  // the same without canonical output
    uint32_t *d_items = nullptr;
    AdvanceDesc *d_adv = nullptr;
    uint32_t n_items = 0;
    FusedShape shape{0, 0};
    bool fused = false;
    int cur = 0;
    hipGraphExec_t graph = nullptr;
    uint32_t graph_sweeps = 64;
    uint64_t graph_key = 0;

    void release() {
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
        for (void *q : {(void *)d_views, (void *)d_views_t, (void *)d_items, (void *)d_adv})
            if (q) (void)hipFree(q);
        d_views = nullptr;
        d_views_t = nullptr;
        d_items = nullptr;
        d_adv = nullptr;
        for (Box *b : boxes) {
            b->in_batch = false;
            b->release();
            delete b;
        }
        boxes.clear();
    }

    // one sweep of every box reading buffer `from`; `canon`: also write the
    // canonical state (the last sweep of a run)
    void launch(int from, uint32_t offset, hipStream_t st, bool canon) {
        if (fused) {
            launch_fused_batch(canon ? d_views : d_views_t, d_items, n_items, (uint32_t)from, offset,
                               shape, st);
        } else {
            for (Box *b : boxes) {
                BoxView v = b->view(from);
                v.offset = offset;
                launch_simple_sweep(v, st);
            }
        }
    }

    int build_items() {
        std::vector<uint32_t> items;
        for (size_t b = 0; b < boxes.size(); ++b) {
            const uint32_t ntx = (boxes[b]->g.M + shape.tile - 1) / shape.tile;
            for (uint32_t t = 0; t < ntx * ntx; ++t) items.push_back(((uint32_t)b << 20) | t);
        }
        if (d_items) (void)hipFree(d_items);
        d_items = nullptr;
        HIPCHK(hipMalloc((void **)&d_items, items.size() * 4));
        HIPCHK(hipMemcpyAsync(d_items, items.data(), items.size() * 4, hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        n_items = (uint32_t)items.size();
        return MPMC_OK;
    }

    uint64_t key() const {
        return ((uint64_t)fused << 60) ^ ((uint64_t)shape.tile << 40) ^
               ((uint64_t)shape.threads << 20) ^ graph_sweeps;
    }

    int build_graph() {
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        for (uint32_t k = 0; k < graph_sweeps; ++k)
            launch((int)(k & 1u), k, cap_stream, k + 1 == graph_sweeps);
        launch_advance_batch(d_adv, (uint32_t)boxes.size(), graph_sweeps, cap_stream);
        HIPCHK(hipStreamEndCapture(cap_stream, &g));
        hipError_t e = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            graph = nullptr;
            return fail(MPMC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        graph_key = key();
        return MPMC_OK;
    }

    int sweep(uint64_t k) {
        for (Box *b : boxes)
            if (b->cur != cur || !b->placed) return fail(MPMC_ESTATE, "batch boxes out of step");
        while (k > 0) {
            if (cur == 0 && k >= graph_sweeps) {
                if (!graph || graph_key != key()) {
                    int rc = build_graph();
                    if (rc) return rc;
                }
                HIPCHK(hipGraphLaunch(graph, stream));
                k -= graph_sweeps;
                continue;
            }
            launch(cur, 0, stream, k == 1);
            launch_advance_batch(d_adv, (uint32_t)boxes.size(), 1, stream);
            HIPCHK(hipGetLastError());
            cur ^= 1;
            --k;
        }
        for (Box *b : boxes) {
            b->cur = cur;
            b->canon_in_c = fused;
        }
        return MPMC_OK;
    }

    // counters of every box
    int read_all(std::vector<DevScalars> &out) {
        out.resize(boxes.size());
        for (size_t b = 0; b < boxes.size(); ++b) {
            int rc = boxes[b]->read_scalars();
            if (rc) return rc;
            out[b] = boxes[b]->host;
        }
        return MPMC_OK;
    }

    // Times `reps` batch launches of a shape; the state in `cur` is only read.
    int time_shape(const FusedShape &s, float *ms) {
        const FusedShape keep = shape;
        const bool keep_fused = fused;
        shape = s;
        fused = true;
        int rc = build_items();
        if (rc) { shape = keep; fused = keep_fused; return rc; }
        for (Box *b : boxes) {
            rc = b->materialize();
            if (rc) { shape = keep; fused = keep_fused; return rc; }
        }
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        for (int r = 0; r < 2; ++r) launch(cur, 0, stream, false);
        (void)hipEventRecord(e0, stream);
        for (int r = 0; r < 6; ++r) launch(cur, 0, stream, false);
        (void)hipEventRecord(e1, stream);
        hipError_t e = hipEventSynchronize(e1);
        float t = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        shape = keep;
        fused = keep_fused;
        if (e != hipSuccess) return fail(MPMC_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
        *ms = t / 6;
        return MPMC_OK;
    }

    int choose(uint32_t tile, uint32_t threads) {
        uint32_t n = 0;
        const FusedShape *shapes = fused_shapes(&n);
        auto fits = [&](const FusedShape &s) {
            for (Box *b : boxes)
                if (!fused_supported(b->view(cur), s)) return false;
            return true;
        };
        if (tile) {
            FusedShape s{tile, threads};
            if (!threads)
                for (uint32_t i = 0; i < n; ++i)
                    if (shapes[i].tile == tile) { s = shapes[i]; break; }
            if (!fits(s)) return fail(MPMC_EINVAL, "shape (%u, %u) does not fit every box", tile, threads);
            shape = s;
            fused = true;
            return build_items();
        }
        std::vector<DevScalars> saved;
        int rc = read_all(saved);
        if (rc) return rc;
        float best = 1e30f;
        bool found = false;
        FusedShape bs{0, 0};
        for (uint32_t i = 0; i < n; ++i) {
            if (!fits(shapes[i])) continue;
            float ms;
            rc = time_shape(shapes[i], &ms);
            if (rc) return rc;
            if (ms < best) { best = ms; bs = shapes[i]; found = true; }
        }
        for (size_t b = 0; b < boxes.size(); ++b) {
            HIPCHK(hipMemcpyAsync(boxes[b]->dev, &saved[b], sizeof(DevScalars), hipMemcpyHostToDevice,
                                  stream));
            boxes[b]->host = saved[b];
        }
        HIPCHK(hipStreamSynchronize(stream));
        if (!found) {
            fused = false;
            shape = FusedShape{0, 0};
            return MPMC_OK;
        }
        shape = bs;
        fused = true;
        return build_items();
    }
};

Batch *BT(mpmc_batch b) { return reinterpret_cast<Batch *>(b); }
}  // namespace

extern "C" int mpmc_batch_create(mpmc_batch *out, uint32_t nbox, const uint32_t *N, const double *eta,
                                 const uint64_t *seed, const mpmc_params *pp) {
    if (!out || !N || !eta || !seed || nbox == 0 || nbox >= 4096)
        return fail(MPMC_EINVAL, "bad batch arguments (1 <= nbox < 4096, arrays non-NULL)");
    *out = nullptr;
    mpmc_params p;
    mpmc_default_params(&p);
    if (pp) p = *pp;
    if (p.alloc) return fail(MPMC_EINVAL, "batches allocate with hipMalloc (no allocator hook)");
    Batch *bt = new Batch();
    bt->p = p;
    bt->stream = (hipStream_t)p.stream;
    for (uint32_t b = 0; b < nbox; ++b) {
        Box *box = nullptr;
        mpmc_params q = p;
        q.schedule = MPMC_SCHED_SIMPLE;
        int rc = create_box(&box, N[b], eta[b], seed[b], &q);
        if (rc) {
            bt->release();
            delete bt;
            return rc;
        }
        box->in_batch = true;
        bt->boxes.push_back(box);
    }
    hipError_t e = hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking);
    std::vector<BoxView> views(2 * nbox), views_t(2 * nbox);
    std::vector<AdvanceDesc> adv(nbox);
    for (uint32_t b = 0; b < nbox; ++b) {
        views[2 * b] = bt->boxes[b]->view(0);
        views[2 * b + 1] = bt->boxes[b]->view(1);
        for (int k = 0; k < 2; ++k) {
            BoxView t = views[2 * b + k];
            t.cnt_can = nullptr;
            t.x_can = t.y_can = nullptr;
            t.tag_can = nullptr;
            views_t[2 * b + k] = t;
        }
        const Box *x = bt->boxes[b];
        adv[b] = AdvanceDesc{x->dev, (uint32_t)x->seed, (uint32_t)(x->seed >> 32), (uint32_t)x->g.W,
                             x->g.Lq};
    }
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_views, views.size() * sizeof(BoxView));
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_views_t, views.size() * sizeof(BoxView));
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_adv, adv.size() * sizeof(AdvanceDesc));
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->d_views, views.data(), views.size() * sizeof(BoxView),
                           hipMemcpyHostToDevice, bt->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->d_views_t, views_t.data(), views_t.size() * sizeof(BoxView),
                           hipMemcpyHostToDevice, bt->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->d_adv, adv.data(), adv.size() * sizeof(AdvanceDesc),
                           hipMemcpyHostToDevice, bt->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);
    if (e != hipSuccess) {
        bt->release();
        delete bt;
        return fail(MPMC_EDEVICE, "batch set-up: %s", hipGetErrorString(e));
    }
    const bool placed = p.lattice != MPMC_LATTICE_NONE;
    int rc = MPMC_OK;
    if (placed && p.schedule != MPMC_SCHED_SIMPLE) rc = bt->choose(p.tile, 0);
    if (rc) {
        bt->release();
        delete bt;
        return rc;
    }
    *out = reinterpret_cast<mpmc_batch>(bt);
    return MPMC_OK;
}

extern "C" int mpmc_batch_free(mpmc_batch b) {
    if (!b) return MPMC_OK;
    (void)hipStreamSynchronize(BT(b)->stream);
    BT(b)->release();
    delete BT(b);
    return MPMC_OK;
}

extern "C" int mpmc_batch_sweep(mpmc_batch bh, uint64_t k, uint64_t *trials, uint64_t *accepts) {
    if (!bh) return fail(MPMC_EINVAL, "NULL batch");
    Batch *b = BT(bh);
    std::vector<DevScalars> before, after;
    if (trials || accepts) {
        int rc = b->read_all(before);
        if (rc) return rc;
    }
    int rc = b->sweep(k);
    if (rc) return rc;
    if (trials || accepts) {
        rc = b->read_all(after);
        if (rc) return rc;
        uint64_t t = 0, a = 0;
        for (size_t i = 0; i < after.size(); ++i) {
            t += after[i].trials - before[i].trials;
            a += after[i].accepts - before[i].accepts;
        }
        if (trials) *trials = t;
        if (accepts) *accepts = a;
    }
    return MPMC_OK;
}

extern "C" int mpmc_batch_box(mpmc_batch bh, uint32_t i, mpmc_box *out) {
    if (!bh || !out) return fail(MPMC_EINVAL, "NULL argument");
    Batch *b = BT(bh);
    if (i >= b->boxes.size()) return fail(MPMC_EINVAL, "box index %u out of range", i);
    *out = reinterpret_cast<mpmc_box>(b->boxes[i]);
    return MPMC_OK;
}

extern "C" int mpmc_batch_accumulate_contacts(mpmc_batch bh) {
    if (!bh) return fail(MPMC_EINVAL, "NULL batch");
    for (Box *x : BT(bh)->boxes) {
        int rc = mpmc_accumulate_contacts(reinterpret_cast<mpmc_box>(x));
        if (rc) return rc;
    }
    return MPMC_OK;
}

extern "C" int mpmc_batch_measure_pressure(mpmc_batch bh, double *p_star, double *se) {
    if (!bh) return fail(MPMC_EINVAL, "NULL batch");
    Batch *b = BT(bh);
    for (size_t i = 0; i < b->boxes.size(); ++i) {
        double P = NAN, s = NAN;
        int rc = mpmc_measure_pressure(reinterpret_cast<mpmc_box>(b->boxes[i]), &P, nullptr, nullptr, &s);
        if (rc) return rc;
        if (p_star) p_star[i] = P;
        if (se) se[i] = s;
    }
    return MPMC_OK;
}

extern "C" int mpmc_batch_set_schedule(mpmc_batch bh, uint32_t tile, uint32_t threads) {
    if (!bh) return fail(MPMC_EINVAL, "NULL batch");
    Batch *b = BT(bh);
    if (tile == 0 && threads == 1) {  // per-box simple kernels
        b->fused = false;
        b->shape = FusedShape{0, 0};
        return MPMC_OK;
    }
    return b->choose(tile, threads);
}

extern "C" int mpmc_batch_info(mpmc_batch bh, uint32_t *nbox, uint32_t *tile, uint32_t *threads,
                               uint32_t *n_items) {
    if (!bh) return fail(MPMC_EINVAL, "NULL batch");
    Batch *b = BT(bh);
    if (nbox) *nbox = (uint32_t)b->boxes.size();
    if (tile) *tile = b->fused ? b->shape.tile : 0;
    if (threads) *threads = b->fused ? b->shape.threads : 0;
    if (n_items) *n_items = b->fused ? b->n_items : 0;
    return MPMC_OK;
}

extern "C" int mpmc_batch_set_graphs(mpmc_batch bh, uint32_t sweeps_per_graph) {
    if (!bh) return fail(MPMC_EINVAL, "NULL batch");
    if (sweeps_per_graph == 0 || (sweeps_per_graph & 1u))
        return fail(MPMC_EINVAL, "sweeps per graph must be even and positive");
    BT(bh)->graph_sweeps = sweeps_per_graph;
    return MPMC_OK;
}
