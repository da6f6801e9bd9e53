// mpmc_host.hpp — host-side state of one box (behind the opaque mpmc_box).
#pragma once
#include <stdarg.h>

#include <vector>

#include "../../include/mpmc.h"
#include "mpmc_kernels.hpp"

namespace mpmc {

// Records a message for mpmc_last_error() and returns code.
int fail(int code, const char *fmt, ...);

struct Geometry {
    double L;      // nominal side sqrt(N pi / eta)
    uint32_t M;    // cells per side
    int64_t W;     // cell width in q units
    float w;       // cell width (exact fp32)
    int64_t Lq;    // simulated side M W in q units
    uint32_t cap;  // disks a cell can hold
    uint32_t CS;   // slots allocated per cell (4 or 8), stored slot-major
};

int compute_geometry(Geometry *g, uint32_t N, double eta, double cell_min, uint32_t step_m);
int build_cells(const Geometry &g, uint32_t N, const int64_t *X, const int64_t *Y,
                std::vector<uint8_t> &hc, std::vector<uint32_t> &ht, std::vector<float> &hx,
                std::vector<float> &hy);

// One set of SoA cell lists (slot-major x, y, tag).
struct CellBuf {
    uint8_t *cnt = nullptr;
    uint32_t *tag = nullptr;
    float *x = nullptr, *y = nullptr;
};

struct Box {
    uint32_t N = 0;
    double eta = 0;
    uint64_t seed = 0;
    mpmc_params p{};
    Geometry g{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    // P[cur]: the cell lists the next sweep reads, already binned in its
    // shifted grid; P[cur ^ 1]: the other buffer.  The canonical state (the
    // box after its last sweep, in that sweep's grid) is C when canon_in_c,
    // else P[cur ^ 1]: the last sweep's input, updated in place by the
    // simple and learned schedules.
    CellBuf P[2], C;
    int cur = 0;
    bool canon_in_c = true;
    CellBuf canon() const { return canon_in_c ? C : P[cur ^ 1]; }
    int materialize();  // moves the canonical state into C
    bool placed = true;
    DevScalars *dev = nullptr;
    DevScalars host{};
    unsigned long long *hist = nullptr;  // ordered pair counts
    float *edges = nullptr;
    uint32_t *scratch_u32 = nullptr;
    void *pos_scratch[2] = {nullptr, nullptr};
    float *psi_buf = nullptr;  // re[N], im[N], field re/im[M*M], by cell slot re/im[CS*M*M]
    int psi_work();            // allocates psi_buf on first use
    uint32_t *loc = nullptr;   // slot of every disk by tag (measurement kernels)
    int locate();              // fills loc for the current state
    void *meas_work = nullptr;  // partial results of the tiled measurement kernels
    void *pos_work = nullptr;   // positional-order partials and staging
    size_t pos_work_bytes = 0;
    int pos_work_at_least(size_t bytes);  // grows pos_work (contents lost)
    float *chi_buf = nullptr;   // chi re/im[N], field re/im[M*M]
    int measure_work();         // allocates meas_work on first use
    uint64_t n_conf = 0;
    // blocks for the pressure standard error
    std::vector<unsigned long long> block_snapshot;
    uint64_t block_conf0 = 0;
    std::vector<double> block_P;
    // schedule
    uint32_t sched = MPMC_SCHED_SIMPLE;
    FusedShape shape{0, 0};
    bool use_graphs = true;
    uint32_t graph_sweeps = 64;
    hipGraphExec_t graph_exec = nullptr;  // all sweeps of a run but the last
    // learned sweeps: a captured run of them, and the learner weights, feature
    // overflow counter and uniform-branch threshold it was captured with
    hipGraphExec_t lgraph_exec = nullptr;
    const void *lgraph_W = nullptr, *lgraph_over = nullptr;
    uint64_t lgraph_E = 0;
    uint32_t lgraph_cpw = 0;
    uint32_t learned_cpw = 0;  // active cells per wave of the learned pass; 0: automatic
    // Asynchronous measurement: its kernels run on meas_stream and read only
    // the canonical buffers C; every later write of C, and every other use of
    // the measurement buffers, first waits for ev_meas on the box's stream.
    hipStream_t meas_stream = nullptr;
    hipEvent_t ev_swept = nullptr, ev_meas = nullptr;
    bool meas_pending = false;
    // [0]: OR of the neighbour-search failures since the last wait (of the
    // widest pass); [1]: the narrower first pass's flag of one measurement
    uint32_t *async_fail = nullptr;
    int join_meas();                 // orders the box's stream after a pending measurement
    int measure_async(double *Psi_dev, bool field);
    uint64_t graph_key = 0;
    uint64_t host_sweeps = 0;
    bool in_batch = false;  // owned by a batch: swept and freed by it
    std::vector<void *> allocations;

    int alloc_dev(void **ptr, size_t bytes);
    void free_dev(void *ptr);  // releases one allocation of alloc_dev
    void release();
    BoxView view(int from) const;
    MeasureView mview() const;
    int sync();
    int read_scalars();
    int upload(const std::vector<uint8_t> &hc, const std::vector<uint32_t> &ht,
               const std::vector<float> &hx, const std::vector<float> &hy, const DevScalars &s);
    // one sweep reading P[from]; `canon`: also write the canonical state
    int launch_one(int from, uint32_t offset, hipStream_t st, bool canon);
    int build_graph();
    uint64_t key() const;
    int run_sweeps(uint64_t k);
    int choose_schedule();
    void *scratch_pos(int which);
};

int create_box(Box **out, uint32_t N, double eta, uint64_t seed, const mpmc_params *p);

// Unweighted least-squares polynomial of `order` through (t_k, y_k), by
// Householder QR; returns 0 and the coefficients, or -1 if singular.
int lsq_poly(const std::vector<double> &t, const std::vector<double> &yv, uint32_t order,
             double *coef);

}  // namespace mpmc
