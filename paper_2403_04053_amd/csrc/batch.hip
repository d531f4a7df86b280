// Batched solves: many independent scattering problems (incident directions,
// energies, potentials, uneven grids) advanced together.  Per axis, the
// instances are grouped by compiled tile shape; one launch covers every
// instance of a group (the workgroups look up their instance from a prefix
// table of tiles), and each instance's step counter lives in device memory,
// so whole groups of steps are captured once in a HIP graph and replayed.
// An instance whose own step count is reached does no further work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "solver.hpp"

namespace {

constexpr int kBatchGraphSteps = 8;

thread_local std::string g_batch_error;

struct Group {
    int variant = 0;
    bool seg = false;
    int potx = 0;       // x and z passes: where the members take the potential term
    std::vector<int> members;
    pstd::PassArgs* d_desc = nullptr;
    int* d_off = nullptr;
    int tiles = 0;
};

}  // namespace

struct pstd_batch {
    std::vector<pstd_solver*> inst;
    hipStream_t stream = nullptr;
    int64_t* ctr = nullptr;  // [count][2]: step, end
    std::vector<Group> groups[3];
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<int> gen;  // table generation of each instance when the groups were built
    int nt = 0;            // an instance's fields outgrow the Infinity Cache
    std::string err;
};

namespace {

pstd_status bfail(pstd_batch* b, pstd_status st, const std::string& m) {
    if (b) b->err = m;
    else g_batch_error = m;
    return st;
}

pstd_status bhip(pstd_batch* b, hipError_t e, const char* what) {
    return bfail(b, e == hipErrorOutOfMemory ? PSTD_ENOMEM : PSTD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIP_TRY(b, call)                                    \
    do {                                                     \
        hipError_t _e = (call);                              \
        if (_e != hipSuccess) return bhip((b), _e, #call);   \
    } while (0)

void free_groups(pstd_batch* b) {
    for (auto& gs : b->groups) {
        for (auto& g : gs) {
            (void)hipFree(g.d_desc);
            (void)hipFree(g.d_off);
        }
        gs.clear();
    }
}

void drop_graph(pstd_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

// (re)build the per-axis launch groups from the instances' current tile
// shapes and tables
pstd_status build_groups(pstd_batch* b) {
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    drop_graph(b);  // the graph holds the old descriptor buffers
    free_groups(b);
    b->gen.resize(b->inst.size());
    // non-temporal z-pass loads when an instance alone outgrows the Infinity
    // Cache (as for a single solve); for many instances that each fit, the
    // hint measured slower (64 instances of 96-192 per axis: 59.0 -> 57.6
    // Gcell/s)
    double largest = 0;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        b->gen[i] = b->inst[i]->tab_gen;
        const pstd_problem& p = b->inst[i]->prob;
        largest = std::max(largest, 24.0 * p.n[0] * p.n[1] * p.n[2]);
    }
    b->nt = largest > pstd::kInfinityCacheBytes ? 1 : 0;
    for (int axis = 0; axis < 3; ++axis) {
        std::vector<Group>& gs = b->groups[axis];
        for (int i = 0; i < (int)b->inst.size(); ++i) {
            const pstd_solver* s = b->inst[i];
            const bool seg = s->prob.sub_core[axis] > 0;
            const int potx = axis == 1 ? 0 : s->potx;
            auto it = std::find_if(gs.begin(), gs.end(), [&](const Group& g) {
                return g.variant == s->variant[axis] && g.seg == seg && g.potx == potx;
            });
            if (it == gs.end()) {
                gs.push_back(Group{});
                it = gs.end() - 1;
                it->variant = s->variant[axis];
                it->seg = seg;
                it->potx = potx;
            }
            it->members.push_back(i);
        }
        for (Group& g : gs) {
            std::vector<pstd::PassArgs> desc(g.members.size());
            std::vector<int> off(g.members.size() + 1, 0);
            for (size_t k = 0; k < g.members.size(); ++k) {
                pstd::solver_args(b->inst[g.members[k]], axis, desc[k]);
                off[k + 1] = off[k] + desc[k].tiles;
            }
            g.tiles = off.back();
            BHIP_TRY(b, hipMalloc(&g.d_desc, desc.size() * sizeof(pstd::PassArgs)));
            BHIP_TRY(b, hipMalloc(&g.d_off, off.size() * sizeof(int)));
            BHIP_TRY(b, hipMemcpy(g.d_desc, desc.data(), desc.size() * sizeof(pstd::PassArgs), hipMemcpyHostToDevice));
            BHIP_TRY(b, hipMemcpy(g.d_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
        }
    }
    return PSTD_OK;
}

// `count` consecutive steps of every instance, then one counter advance
pstd_status launch_batch_steps(pstd_batch* b, hipStream_t stream, int count) {
    for (int k = 0; k < count; ++k)
        for (int axis = 0; axis < 3; ++axis)
            for (const Group& g : b->groups[axis]) {
                hipError_t e = pstd::launch_variant(g.variant, g.seg, axis, g.d_desc, g.d_off, (int)g.members.size(),
                                                    g.tiles, k, g.potx, b->nt, stream);
                if (e != hipSuccess) return bhip(b, e, "batch pass launch");
            }
    hipError_t e = pstd::launch_advance(b->ctr, (int)b->inst.size(), count, stream);
    if (e != hipSuccess) return bhip(b, e, "batch advance");
    return PSTD_OK;
}

pstd_status build_batch_graph(pstd_batch* b) {
    if (b->graph) return PSTD_OK;
    if (!b->cap_stream) BHIP_TRY(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    BHIP_TRY(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    pstd_status st = launch_batch_steps(b, b->cap_stream, kBatchGraphSteps);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return bhip(b, e, "batch graph capture");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return bhip(b, e, "batch graph instantiate");
    }
    return PSTD_OK;
}

}  // namespace

extern "C" {

pstd_status pstd_batch_create(const pstd_problem* problems, int32_t count, void* hip_stream, pstd_batch** out) {
    if (!problems || !out || count < 1) return PSTD_EINVAL;
    *out = nullptr;
    pstd_batch* b = new pstd_batch();
    b->stream = (hipStream_t)hip_stream;
    hipError_t e = hipMalloc(&b->ctr, 2 * sizeof(int64_t) * count);
    if (e) {
        delete b;
        return bhip(nullptr, e, "hipMalloc counters");
    }
    for (int i = 0; i < count; ++i) {
        pstd_solver* s = nullptr;
        pstd_status st = pstd::solver_create(&problems[i], b->stream, b->ctr + 2 * i, &s);
        if (st) {
            std::string m = "instance " + std::to_string(i) + ": " + pstd_last_error(nullptr);
            pstd_batch_destroy(b);
            return bfail(nullptr, st, m);
        }
        b->inst.push_back(s);
    }
    pstd_status st = build_groups(b);
    if (st) {
        std::string m = b->err;
        pstd_batch_destroy(b);
        return bfail(nullptr, st, m);
    }
    *out = b;
    return PSTD_OK;
}

pstd_status pstd_batch_size(const pstd_batch* b, int32_t* count_out) {
    if (!b || !count_out) return PSTD_EINVAL;
    *count_out = (int32_t)b->inst.size();
    return PSTD_OK;
}

pstd_status pstd_batch_solver(pstd_batch* b, int32_t idx, pstd_solver** out) {
    if (!b || !out || idx < 0 || idx >= (int32_t)b->inst.size()) return PSTD_EINVAL;
    *out = b->inst[idx];
    return PSTD_OK;
}

pstd_status pstd_batch_set_potential(pstd_batch* b, int32_t idx, const float* V_dev, int64_t n_cells) {
    if (!b || idx < 0 || idx >= (int32_t)b->inst.size()) return PSTD_EINVAL;
    pstd_status st = pstd_set_potential(b->inst[idx], V_dev, n_cells);
    if (st) return bfail(b, st, "instance " + std::to_string(idx) + ": " + b->inst[idx]->err);
    return PSTD_OK;
}

pstd_status pstd_batch_autotune(pstd_batch* b, int32_t reps) {
    if (!b || reps < 1) return PSTD_EINVAL;
    // tune the largest instance of every distinct (axis pass) length and share
    // its choice with the instances of that length
    for (int axis = 0; axis < 3; ++axis) {
        std::vector<std::pair<int, int>> done;  // (local length, variant)
        std::vector<int> order(b->inst.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return b->inst[x]->cells > b->inst[y]->cells; });
        for (int i : order) {
            pstd_solver* s = b->inst[i];
            const int len = s->prob.sub_core[axis] > 0 ? s->prob.sub_core[axis] + 2 * s->prob.sub_halo : s->prob.n[axis];
            auto it = std::find_if(done.begin(), done.end(), [&](const std::pair<int, int>& d) { return d.first == len; });
            if (it != done.end()) {
                s->variant[axis] = it->second;
                continue;
            }
            pstd_status st = pstd::solver_autotune(s, reps);
            if (st) return bfail(b, st, s->err);
            done.push_back({len, s->variant[axis]});
        }
    }
    drop_graph(b);
    return build_groups(b);
}

pstd_status pstd_batch_run(pstd_batch* b, const int64_t* n_steps_host) {
    if (!b || !n_steps_host) return PSTD_EINVAL;
    const int count = (int)b->inst.size();
    std::vector<int64_t> c(2 * count);
    int64_t most = 0;
    bool grew = false;
    for (int i = 0; i < count; ++i) {
        if (n_steps_host[i] < 0) return bfail(b, PSTD_EINVAL, "negative step count");
        pstd_solver* s = b->inst[i];
        pstd_status st = pstd::solver_ensure_tables(s, s->step + n_steps_host[i]);
        if (st) return bfail(b, st, s->err);
        grew |= s->tab_gen != b->gen[i];
        c[2 * i] = s->step;
        c[2 * i + 1] = s->step + n_steps_host[i];
        most = std::max(most, n_steps_host[i]);
    }
    if (grew) {
        pstd_status st = build_groups(b);
        if (st) return st;
    }
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    BHIP_TRY(b, hipMemcpy(b->ctr, c.data(), c.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    int64_t left = most;
    if (left >= kBatchGraphSteps) {
        pstd_status st = build_batch_graph(b);
        if (st) return st;
        for (; left >= kBatchGraphSteps; left -= kBatchGraphSteps) BHIP_TRY(b, hipGraphLaunch(b->graph, b->stream));
    }
    if (left > 0) {
        pstd_status st = launch_batch_steps(b, b->stream, (int)left);
        if (st) return st;
    }
    for (int i = 0; i < count; ++i) {
        pstd_solver* s = b->inst[i];
        pstd::solver_account_steps(s, s->step, s->step + n_steps_host[i]);
        s->step += n_steps_host[i];
    }
    return PSTD_OK;
}

pstd_status pstd_batch_destroy(pstd_batch* b) {
    if (!b) return PSTD_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    free_groups(b);
    for (pstd_solver* s : b->inst) pstd_destroy(s);
    (void)hipFree(b->ctr);
    delete b;
    return PSTD_OK;
}

const char* pstd_batch_last_error(const pstd_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"
