// Batched applies of independent problems: every tree of a batch applies V_h
// to its own density in one stream-ordered call.  The per-problem applies
// (the stages of Algorithm 2 for one tree) are captured once into a HIP
// graph whose branches run on separate streams, so small problems overlap
// each other and the large ones instead of queueing one after another.  When
// trees have levels with unequal intervals (the class-aware M2L), the M2L of
// those levels of all trees runs as one cross-problem launch per (precision,
// time offset) between the trees' upward and downward passes; the
// graph is replayed for every further call with the same vectors and tree
// precisions, and re-captured when either changes.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "internal.hpp"
#include "pfmm.h"

using namespace pfmm;

struct pfmm_batch {
    int device = 0;
    std::vector<pfmm_tree*> trees;
    std::vector<hipStream_t> streams;      // branch streams (default priority)
    hipStream_t cap = nullptr;             // the stream the graph is captured on (never the caller's:
                                           // the legacy default stream cannot be captured)
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const double*> key_w;      // vectors the graph was captured with
    std::vector<double*> key_f;
    std::vector<int> key_prec;             // each tree's farfield precision at capture (the graph
                                           // holds that precision's kernels and tables)
    BatchM2L* xm = nullptr;                // cross-problem M2L of the levels with unequal intervals
    bool use_xm = true;
};

namespace {

constexpr int kMaxBranches = 8;

#define HIP_CHECK(expr)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return set_error(PFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

void release_graph(pfmm_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->key_w.clear();
    b->key_f.clear();
    b->key_prec.clear();
}

// Capture the applies of all trees into b->graph / b->exec (recorded on the
// batch's own stream, nothing runs).  Tree i runs on branch stream
// i mod branches, in batch order, forked from and joined back into the
// capture stream; the graph is then launched on the caller's stream.
pfmm_status capture(pfmm_batch* b, const double* const* w, double* const* f) {
    release_graph(b);
    hipStream_t st = b->cap;
    const bool xm = b->xm && b->use_xm;
    if (xm) {
        const pfmm_status ps = batch_m2l_prepare(b->xm);   // unit descriptors for the current precisions
        if (ps != PFMM_OK) return ps;
    }
    HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    pfmm_status status = PFMM_OK;
    hipError_t e = hipSuccess;
    const int nb = (int)b->streams.size();
    // fork the branch streams from st, run `body(tree, stream)` for every
    // tree on branch i mod nb, join them back into st
    auto branches = [&](auto body) {
        if (e == hipSuccess) e = hipEventRecord(b->fork, st);
        for (int s = 0; s < nb && e == hipSuccess; ++s) e = hipStreamWaitEvent(b->streams[s], b->fork, 0);
        for (size_t i = 0; i < b->trees.size() && e == hipSuccess && status == PFMM_OK; ++i)
            status = body(i, b->streams[i % nb]);
        for (int s = 0; s < nb && e == hipSuccess; ++s) {
            e = hipEventRecord(b->joins[s], b->streams[s]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, b->joins[s], 0);
        }
    };
    if (!xm) {
        branches([&](size_t i, hipStream_t sb) { return tree_apply(b->trees[i], false, w[i], f[i], sb); });
    } else {
        // upward passes and nearfields per tree, one M2L launch per (precision,
        // time offset) for the levels with unequal intervals of all trees,
        // then the downward passes per tree
        branches([&](size_t i, hipStream_t sb) { return tree_apply_phase(b->trees[i], false, w[i], f[i], sb, 1); });
        if (e == hipSuccess && status == PFMM_OK) status = batch_m2l_launch(b->xm, st);
        branches([&](size_t i, hipStream_t sb) { return tree_apply_phase(b->trees[i], false, w[i], f[i], sb, 2); });
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &g);
    if (status != PFMM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return status;
    }
    if (e != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_error(PFMM_EDEVICE, std::string("batch capture failed: ") +
                                           hipGetErrorString(e != hipSuccess ? e : ee));
    }
    b->graph = g;
    HIP_CHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->key_w.assign(w, w + b->trees.size());
    b->key_f.assign(f, f + b->trees.size());
    b->key_prec.resize(b->trees.size());
    for (size_t i = 0; i < b->trees.size(); ++i) b->key_prec[i] = tree_precision(b->trees[i]);
    return PFMM_OK;
}

}  // namespace

extern "C" {

pfmm_status pfmm_batch_create(pfmm_tree* const* trees, int32_t n, pfmm_batch** out) {
    if (!out) return set_error(PFMM_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (!trees || n < 1) return set_error(PFMM_EINVAL, "empty batch");
    for (int i = 0; i < n; ++i) {
        if (!trees[i]) return set_error(PFMM_EINVAL, "NULL tree in batch");
        if (!tree_has(trees[i], PFMM_OP_V)) return set_error(PFMM_EINVAL, "a tree of the batch holds no V_h");
        if (tree_device(trees[i]) != tree_device(trees[0]))
            return set_error(PFMM_EINVAL, "the trees of a batch must live on one device");
        for (int j = 0; j < i; ++j)
            if (trees[j] == trees[i]) return set_error(PFMM_EINVAL, "a tree appears twice in the batch");
    }
    pfmm_batch* b = new (std::nothrow) pfmm_batch();
    if (!b) return set_error(PFMM_ENOMEM, "host allocation failed");
    b->device = tree_device(trees[0]);
    b->trees.assign(trees, trees + n);
    if (hipSetDevice(b->device) != hipSuccess) {
        delete b;
        return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    }
    const int nb = n < kMaxBranches ? n : kMaxBranches;
    b->streams.assign(nb, nullptr);
    b->joins.assign(nb, nullptr);
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int s = 0; s < nb && e == hipSuccess; ++s) {
        e = hipStreamCreateWithFlags(&b->streams[s], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->joins[s], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        pfmm_batch_destroy(b);
        return set_error(PFMM_EDEVICE, std::string("batch streams: ") + hipGetErrorString(e));
    }
    const pfmm_status xs = batch_m2l_create(trees, n, &b->xm);
    if (xs != PFMM_OK) {
        pfmm_batch_destroy(b);
        return xs;
    }
    *out = b;
    return PFMM_OK;
}

pfmm_status pfmm_apply_V_batch(pfmm_batch* b, const double* const* w_dev, double* const* f_dev, void* stream) {
    if (!b || !w_dev || !f_dev) return set_error(PFMM_EINVAL, "NULL argument");
    const size_t n = b->trees.size();
    for (size_t i = 0; i < n; ++i) {
        if (!w_dev[i] || !f_dev[i]) return set_error(PFMM_EINVAL, "NULL vector in batch");
        if (tree_profiling(b->trees[i])) return set_error(PFMM_EINVAL, "stage profiling is on for a tree of the batch");
    }
    if (hipSetDevice(b->device) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    bool same = b->exec != nullptr;
    for (size_t i = 0; same && i < n; ++i)
        same = b->key_w[i] == w_dev[i] && b->key_f[i] == f_dev[i] && b->key_prec[i] == tree_precision(b->trees[i]);
    if (!same) {
        const pfmm_status s = capture(b, w_dev, f_dev);
        if (s != PFMM_OK) return s;
    }
    HIP_CHECK(hipGraphLaunch(b->exec, st));
    return PFMM_OK;
}

pfmm_status pfmm_batch_set_cross_m2l(pfmm_batch* b, int32_t enable) {
    if (!b) return set_error(PFMM_EINVAL, "NULL batch");
    if ((enable != 0) != b->use_xm) {
        b->use_xm = enable != 0;
        release_graph(b);   // the next apply re-captures
    }
    return PFMM_OK;
}

void pfmm_batch_destroy(pfmm_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    release_graph(b);
    batch_m2l_destroy(b->xm);
    for (hipStream_t s : b->streams)
        if (s) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipEvent_t e : b->joins)
        if (e) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

}  // extern "C"
