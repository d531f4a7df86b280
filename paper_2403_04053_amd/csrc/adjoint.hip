// Fresnel-plane intensity misfit and its gradient with respect to the voxel
// potential by the discrete adjoint of the leapfrog scheme (Eq. PSTDupdating),
// of the surface DFT (Eqs. psiphasor, dpsiphasor, scaledphsiphasor) and of
// the box projection (Section 3.2).
//
// Forward: from rest, n_steps steps; at the start of every segment of S
// steps the pair (psi^{kS-1}, psi^{kS}) is copied aside (ceil(n_steps / S)
// checkpoints).  The surface phasors are projected to the observation points
// and J = 1/2 sum_o (|exp(i khat . r_o) + Psi_o|^2 - I_o)^2 is formed in FP64.
//
// Backward, segments last to first:
//   - restore the segment's checkpoint and recompute its states with the
//     surface DFT switched off, each step also storing psi^{n+1} in the
//     segment store;
//   - run the adjoint steps of the segment.  With chi^m = conj(Gamma mu^m)
//     (mu the Lagrange multipliers of the step equations) the recurrence is
//       chi^m = Gamma (chi^{m+2} - i [A chi^{m+1} + i conj(e_m)]),
//     A = 2 dtau (eta K + V / E0), the same passes as a forward step with no
//     incident source; conj(e_m) = w_m conj(B^H h) / Phi_inc is injected
//     along each pencil through the two derivative rows of its axis
//     (h = G^H g: the projection adjoint of the seed g_o = r_o T_o);
//   - the z pass accumulates Im(chi^m psi^{m-1}) per cell in FP32; the sum
//     is folded into an FP64 accumulator at the end of every segment.
// dJ/dV = (4 dtau / E0) sum_m Im(chi^m psi^{m-1}).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "solver.hpp"

namespace pstd {

struct AdjointState {
    int64_t N = 0;        // forward steps of the misfit run
    int64_t S = 0;        // segment length
    int64_t nck = 0;      // segments
    int64_t cells = 0;
    float2* ck = nullptr;       // [nck][2][cells]: psi^{kS-1}, psi^{kS}
    float2* last = nullptr;     // [2][cells]: psi^{N-1}, psi^N
    float2* store = nullptr;    // [S-1][cells]: psi^{kS+1} .. psi^{kS+S-1}
    float2* chi[2] = {nullptr, nullptr};
    float* g32 = nullptr;
    double* g64 = nullptr;
    int64_t n_obs = 0;
    double3* obs = nullptr;
    double* target = nullptr;
    double2* psi_obs = nullptr;  // scattered Psi at the points
    double2* seed = nullptr;     // g_o = (|T_o|^2 - I_o) T_o
    double* J = nullptr;
    float2* inj = nullptr;       // conj(G^H g) / Phi_inc, phasor layout
    // step tables
    int* dft_off = nullptr;              // [N] zeros: recompute steps skip the DFT
    float2** stash = nullptr;            // [N] recompute: where psi^{n+1} goes
    double2* w_adj = nullptr;            // [N] i exp(i tau_m), m = N - k
    int* dft_adj = nullptr;              // [N] m inside the window
    const float2** fwd_adj = nullptr;    // [N] psi^{m-1}
    int64_t* ctr_adj = nullptr;
    bool valid = false;                  // a forward run matches the solver state
};

}  // namespace pstd

namespace {

using pstd::AdjointState;

constexpr int kAdjGraphSteps = 16;

pstd_status fail(pstd_solver* s, pstd_status st, const std::string& m) { return pstd::solver_fail(s, st, m); }
pstd_status hfail(pstd_solver* s, hipError_t e, const char* what) { return pstd::solver_hip_fail(s, e, what); }

#define ADJ_TRY(s, call)                                    \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return hfail((s), _e, #call); \
    } while (0)

void free_adjoint(AdjointState* a) {
    if (!a) return;
    void* ptrs[] = {a->ck,     a->last,   a->store,   a->chi[0], a->chi[1], a->g32,     a->g64,
                    a->obs,    a->target, a->psi_obs, a->seed,   a->J,      a->inj,     a->dft_off,
                    a->stash,  a->w_adj,  a->dft_adj, (void*)a->fwd_adj,     a->ctr_adj};
    for (void* p : ptrs) (void)hipFree(p);
    delete a;
}

// misfit terms: T_o = exp(i khat . k0 r_o) + Psi_o, r_o = |T_o|^2 - I_o,
// seed g_o = r_o T_o, J = 1/2 sum r_o^2 (one workgroup, FP64)
constexpr int kMisfitThreads = 256;

__global__ __launch_bounds__(kMisfitThreads) void misfit_kernel(const double3* __restrict__ obs,
                                                                const double2* __restrict__ psi,
                                                                const double* __restrict__ target, int64_t n,
                                                                double k0, double khx, double khy, double khz,
                                                                double2* __restrict__ seed, double* __restrict__ J) {
    __shared__ double red[kMisfitThreads];
    double acc = 0.0;
    for (int64_t o = threadIdx.x; o < n; o += kMisfitThreads) {
        const double3 r = obs[o];
        const double ph = k0 * (khx * r.x + khy * r.y + khz * r.z);
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double tr = cs + psi[o].x, ti = sn + psi[o].y;
        const double res = tr * tr + ti * ti - target[o];
        seed[o] = make_double2(res * tr, res * ti);
        acc += res * res;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kMisfitThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) J[0] = 0.5 * red[0];
}

// counters (step, end) of one solve, written by one lane
__global__ void set_ctr_kernel(int64_t* ctr, int64_t n, int64_t end) {
    if (threadIdx.x == 0) {
        ctr[0] = n;
        ctr[1] = end;
    }
}

hipError_t set_ctr(int64_t* ctr, int64_t n, int64_t end, hipStream_t stream) {
    hipLaunchKernelGGL(set_ctr_kernel, dim3(1), dim3(64), 0, stream, ctr, n, end);
    return hipGetLastError();
}

// descriptors of the recompute steps (forward passes, no surface DFT, stash)
void recompute_args(const pstd_solver* s, const AdjointState* a, int axis, pstd::PassArgs& pa) {
    pstd::solver_args(s, axis, pa);
    pa.dft_tab = a->dft_off;
    pa.stash_tab = a->stash;
}

// descriptors of the adjoint steps
void adjoint_args(const pstd_solver* s, const AdjointState* a, int axis, pstd::PassArgs& pa) {
    pstd::solver_args(s, axis, pa);
    pa.buf[0] = a->chi[0];
    pa.buf[1] = a->chi[1];
    pa.ctr = a->ctr_adj;
    pa.w_tab = a->w_adj;
    pa.dft_tab = a->dft_adj;
    pa.fwd_tab = a->fwd_adj;
    pa.grad = a->g32;
    pa.acc = nullptr;
    // the phasor layout: face f = 2 axis + side holds (psi plane, dpsi plane)
    const int64_t np = s->points[axis];
    int64_t off = 0;
    for (int f = 0; f < 2 * axis; ++f) off += 2 * s->points[f / 2];
    pa.inj_lo_p = a->inj + off;
    pa.inj_lo_d = a->inj + off + np;
    pa.inj_hi_p = a->inj + off + 2 * np;
    pa.inj_hi_d = a->inj + off + 3 * np;
}

pstd_status launch_rec(pstd_solver* s, AdjointState* a, hipStream_t st, int count) {
    for (int k = 0; k < count; ++k)
        for (int axis = 0; axis < 3; ++axis) {
            pstd::PassArgs pa;
            recompute_args(s, a, axis, pa);
            hipError_t e = pstd::launch_variant_single(s->variant[axis], false, axis, pa, k, st);
            if (e) return hfail(s, e, "recompute pass");
        }
    hipError_t e = pstd::launch_advance(s->ctr, 1, count, st);
    if (e) return hfail(s, e, "advance");
    return PSTD_OK;
}

pstd_status launch_adj(pstd_solver* s, AdjointState* a, hipStream_t st, int count) {
    for (int k = 0; k < count; ++k)
        for (int axis = 0; axis < 3; ++axis) {
            pstd::PassArgs pa;
            adjoint_args(s, a, axis, pa);
            hipError_t e = pstd::launch_variant_adjoint(s->variant[axis], axis, pa, k, st);
            if (e) return hfail(s, e, "adjoint pass");
        }
    hipError_t e = pstd::launch_advance(a->ctr_adj, 1, count, st);
    if (e) return hfail(s, e, "advance");
    return PSTD_OK;
}

template <class F>
pstd_status capture(pstd_solver* s, F&& body, hipGraphExec_t* out) {
    *out = nullptr;
    if (!s->cap_stream) ADJ_TRY(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    ADJ_TRY(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    pstd_status st = body(s->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e) return hfail(s, e, "graph capture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e) {
        *out = nullptr;
        return hfail(s, e, "graph instantiate");
    }
    return PSTD_OK;
}

// `count` steps: whole graphs, then single launches
template <class F>
pstd_status run_steps(pstd_solver* s, hipGraphExec_t graph, int64_t count, F&& eager) {
    int64_t left = count;
    for (; left >= kAdjGraphSteps; left -= kAdjGraphSteps) ADJ_TRY(s, hipGraphLaunch(graph, s->stream));
    if (left > 0) return eager((int)left);
    return PSTD_OK;
}

template <class T>
hipError_t alloc(T** p, size_t count) {
    return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace

namespace pstd {

void adjoint_invalidate(pstd_solver* s) {
    if (s && s->adj) s->adj->valid = false;
}

void adjoint_free(pstd_solver* s) {
    if (!s) return;
    free_adjoint(s->adj);
    s->adj = nullptr;
}

}  // namespace pstd

extern "C" {

pstd_status pstd_misfit_forward(pstd_solver* s, int64_t n_steps, const double* obs_dev, int64_t n_obs,
                                const double* target_dev, int32_t n_checkpoints, double* J_host) {
    if (!s || !obs_dev || !target_dev || !J_host) return PSTD_EINVAL;
    if (s->in_batch) return fail(s, PSTD_ESTATE, "instances of a batch are stepped by the batch");
    if (n_steps < 1 || n_obs < 1) return fail(s, PSTD_EINVAL, "n_steps and n_obs must be positive");
    if (n_checkpoints < 1 || n_checkpoints > n_steps) return fail(s, PSTD_EINVAL, "n_checkpoints must lie in [1, n_steps]");
    if (s->prob.sub_core[0] > 0 || s->prob.sub_core[1] > 0 || s->prob.sub_core[2] > 0)
        return fail(s, PSTD_EUNSUPPORTED, "the adjoint runs on whole-axis pencils only");
    if (s->sphere) return fail(s, PSTD_EUNSUPPORTED, "the misfit projects from the box surface only");
    if (s->prob.scheme != 0) return fail(s, PSTD_EUNSUPPORTED, "the misfit runs the spectral scheme only");
    if (s->pulse) return fail(s, PSTD_EUNSUPPORTED, "the misfit takes the monochromatic wave only");
    if (std::min<int64_t>(s->prob.dft_end, n_steps) <= s->prob.dft_begin)
        return fail(s, PSTD_EINVAL, "no step of the DFT window lies in [0, n_steps)");
    const int64_t S = (n_steps + n_checkpoints - 1) / n_checkpoints;
    const int64_t nck = (n_steps + S - 1) / S;
    const int64_t cells = s->cells;
    AdjointState* a = s->adj;
    if (a && (a->N != n_steps || a->S != S || a->n_obs != n_obs)) {
        ADJ_TRY(s, hipStreamSynchronize(s->stream));
        pstd::adjoint_free(s);
        a = nullptr;
    }
    if (!a) {
        a = new AdjointState();
        s->adj = a;
        a->N = n_steps;
        a->S = S;
        a->nck = nck;
        a->cells = cells;
        a->n_obs = n_obs;
        int64_t inj_n = 0;
        for (int f = 0; f < 6; ++f) inj_n += 2 * s->points[f / 2];
        hipError_t e;
        if ((e = alloc(&a->ck, (size_t)nck * 2 * cells)) || (e = alloc(&a->last, (size_t)2 * cells)) ||
            (e = alloc(&a->store, (size_t)std::max<int64_t>(S - 1, 1) * cells)) ||
            (e = alloc(&a->chi[0], (size_t)cells)) || (e = alloc(&a->chi[1], (size_t)cells)) ||
            (e = alloc(&a->g32, (size_t)cells)) || (e = alloc(&a->g64, (size_t)cells)) ||
            (e = alloc(&a->obs, (size_t)n_obs)) || (e = alloc(&a->target, (size_t)n_obs)) ||
            (e = alloc(&a->psi_obs, (size_t)n_obs)) || (e = alloc(&a->seed, (size_t)n_obs)) ||
            (e = alloc(&a->J, 1)) || (e = alloc(&a->inj, (size_t)inj_n)) || (e = alloc(&a->dft_off, (size_t)n_steps)) ||
            (e = alloc(&a->stash, (size_t)n_steps)) || (e = alloc(&a->w_adj, (size_t)n_steps)) ||
            (e = alloc(&a->dft_adj, (size_t)n_steps)) || (e = alloc(&a->fwd_adj, (size_t)n_steps)) ||
            (e = alloc(&a->ctr_adj, 2))) {
            pstd::adjoint_free(s);
            return hfail(s, e, "hipMalloc adjoint state");
        }
    }
    a->valid = false;
    ADJ_TRY(s, hipMemcpyAsync(a->obs, obs_dev, n_obs * sizeof(double3), hipMemcpyDeviceToDevice, s->stream));
    ADJ_TRY(s, hipMemcpyAsync(a->target, target_dev, n_obs * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    // from rest
    ADJ_TRY(s, hipMemsetAsync(s->buf[0], 0, cells * sizeof(float2), s->stream));
    ADJ_TRY(s, hipMemsetAsync(s->buf[1], 0, cells * sizeof(float2), s->stream));
    for (int ax = 0; ax < 3; ++ax) ADJ_TRY(s, hipMemsetAsync(s->acc[ax], 0, 8 * s->points[ax] * sizeof(double2), s->stream));
    ADJ_TRY(s, set_ctr(s->ctr, 0, std::numeric_limits<int64_t>::max(), s->stream));
    s->step = 0;
    s->inc_sum = 0;
    pstd_status st = pstd::solver_ensure_tables(s, n_steps);
    if (st) return st;
    for (int64_t k = 0; k < nck; ++k) {
        const int64_t n0 = k * S;
        float2* slot = a->ck + (size_t)k * 2 * cells;
        ADJ_TRY(s, hipMemcpyAsync(slot, s->buf[(n0 + 1) & 1], cells * sizeof(float2), hipMemcpyDeviceToDevice, s->stream));
        ADJ_TRY(s, hipMemcpyAsync(slot + cells, s->buf[n0 & 1], cells * sizeof(float2), hipMemcpyDeviceToDevice, s->stream));
        st = pstd_run(s, std::min(S, n_steps - n0));
        if (st) return st;
    }
    ADJ_TRY(s, hipMemcpyAsync(a->last, s->buf[(n_steps + 1) & 1], cells * sizeof(float2), hipMemcpyDeviceToDevice, s->stream));
    ADJ_TRY(s, hipMemcpyAsync(a->last + cells, s->buf[n_steps & 1], cells * sizeof(float2), hipMemcpyDeviceToDevice,
                              s->stream));
    st = pstd_project(s, (const double*)a->obs, n_obs, (double*)a->psi_obs);
    if (st) return st;
    hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(kMisfitThreads), 0, s->stream, a->obs, a->psi_obs, a->target, n_obs,
                       s->prob.k0, s->kh[0], s->kh[1], s->kh[2], a->seed, a->J);
    ADJ_TRY(s, hipGetLastError());
    ADJ_TRY(s, hipMemcpyAsync(J_host, a->J, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    ADJ_TRY(s, hipStreamSynchronize(s->stream));
    if (!std::isfinite(*J_host)) return fail(s, PSTD_ENONFINITE, "misfit is not finite");
    a->valid = true;
    return PSTD_OK;
}

pstd_status pstd_misfit_backward(pstd_solver* s, float* dJdV_dev, int64_t n_cells) {
    if (!s || !dJdV_dev) return PSTD_EINVAL;
    if (n_cells != s->cells) return fail(s, PSTD_EINVAL, "n_cells does not match the grid");
    AdjointState* a = s->adj;
    if (!a || !a->valid || s->step != a->N)
        return fail(s, PSTD_ESTATE, "no misfit forward run matches the solver state");
    const int64_t N = a->N, S = a->S, cells = a->cells;
    // seed of the surface injection: conj(G^H g) / Phi_inc
    {
        std::string msg;
        hipError_t e = pstd::project_adjoint(&s->proj, s->prob, s->dxb, s->acc, s->points, 1.0 / s->inc_sum, a->obs,
                                             a->n_obs, a->seed, a->inj, s->stream, &msg);
        if (e) return msg.empty() ? hfail(s, e, "project_adjoint") : fail(s, PSTD_EINVAL, msg);
    }
    // step tables
    {
        std::vector<int> off(N, 0), on(N);
        std::vector<float2*> stash(N, nullptr);
        std::vector<double2> w(N);
        std::vector<const float2*> fwd(N);
        for (int64_t n = 0; n < N; ++n) {
            const int64_t n0 = (n / S) * S;
            if (n + 1 - n0 < S && n + 1 < N) stash[n] = a->store + (size_t)(n - n0) * cells;
        }
        for (int64_t k = 0; k < N; ++k) {
            const int64_t m = N - k;
            const double tau = m * s->dtau;
            w[k] = make_double2(-std::sin(tau), std::cos(tau));  // i exp(i tau_m)
            on[k] = (m >= s->prob.dft_begin && m < std::min<int64_t>(s->prob.dft_end, N)) ? 1 : 0;
            const int64_t j = m - 1, seg = j / S, j0 = seg * S;
            fwd[k] = j == j0 ? a->ck + ((size_t)seg * 2 + 1) * cells : a->store + (size_t)(j - j0 - 1) * cells;
        }
        ADJ_TRY(s, hipStreamSynchronize(s->stream));
        ADJ_TRY(s, hipMemcpy(a->dft_off, off.data(), N * sizeof(int), hipMemcpyHostToDevice));
        ADJ_TRY(s, hipMemcpy(a->stash, stash.data(), N * sizeof(float2*), hipMemcpyHostToDevice));
        ADJ_TRY(s, hipMemcpy(a->w_adj, w.data(), N * sizeof(double2), hipMemcpyHostToDevice));
        ADJ_TRY(s, hipMemcpy(a->dft_adj, on.data(), N * sizeof(int), hipMemcpyHostToDevice));
        ADJ_TRY(s, hipMemcpy(a->fwd_adj, fwd.data(), N * sizeof(const float2*), hipMemcpyHostToDevice));
    }
    ADJ_TRY(s, hipMemsetAsync(a->chi[0], 0, cells * sizeof(float2), s->stream));
    ADJ_TRY(s, hipMemsetAsync(a->chi[1], 0, cells * sizeof(float2), s->stream));
    ADJ_TRY(s, hipMemsetAsync(a->g32, 0, cells * sizeof(float), s->stream));
    ADJ_TRY(s, hipMemsetAsync(a->g64, 0, cells * sizeof(double), s->stream));
    hipGraphExec_t grec = nullptr, gadj = nullptr;
    auto done = [&](pstd_status st) {
        if (grec) (void)hipGraphExecDestroy(grec);
        if (gadj) (void)hipGraphExecDestroy(gadj);
        return st;
    };
    pstd_status st;
    if ((st = capture(s, [&](hipStream_t cs) { return launch_rec(s, a, cs, kAdjGraphSteps); }, &grec))) return done(st);
    if ((st = capture(s, [&](hipStream_t cs) { return launch_adj(s, a, cs, kAdjGraphSteps); }, &gadj))) return done(st);
    for (int64_t k = a->nck - 1; k >= 0; --k) {
        const int64_t n0 = k * S, n1 = std::min(n0 + S, N);
        // states psi^{n0+1} .. psi^{n1-1} into the segment store
        const int64_t nrec = n1 - 1 - n0;
        if (nrec > 0) {
            const float2* slot = a->ck + (size_t)k * 2 * cells;
            hipError_t e;
            if ((e = hipMemcpyAsync(s->buf[(n0 + 1) & 1], slot, cells * sizeof(float2), hipMemcpyDeviceToDevice,
                                    s->stream)) ||
                (e = hipMemcpyAsync(s->buf[n0 & 1], slot + cells, cells * sizeof(float2), hipMemcpyDeviceToDevice,
                                    s->stream)) ||
                (e = set_ctr(s->ctr, n0, n0 + nrec, s->stream)))
                return done(hfail(s, e, "segment restore"));
            st = run_steps(s, grec, nrec, [&](int c) { return launch_rec(s, a, s->stream, c); });
            if (st) return done(st);
        }
        // adjoint steps m = n1 .. n0 + 1  (k' = N - m)
        hipError_t e = set_ctr(a->ctr_adj, N - n1, N - n0, s->stream);
        if (e) return done(hfail(s, e, "adjoint counters"));
        st = run_steps(s, gadj, n1 - n0, [&](int c) { return launch_adj(s, a, s->stream, c); });
        if (st) return done(st);
        e = pstd::launch_fold(a->g64, a->g32, cells, s->stream);
        if (e) return done(hfail(s, e, "fold"));
    }
    hipError_t e = pstd::launch_scale_out(a->g64, 4.0 * s->dtau / s->E0, dJdV_dev, cells, s->stream);
    if (e) return done(hfail(s, e, "gradient"));
    // back to the state at the end of the forward run
    if ((e = hipMemcpyAsync(s->buf[(N + 1) & 1], a->last, cells * sizeof(float2), hipMemcpyDeviceToDevice, s->stream)) ||
        (e = hipMemcpyAsync(s->buf[N & 1], a->last + cells, cells * sizeof(float2), hipMemcpyDeviceToDevice,
                            s->stream)) ||
        (e = set_ctr(s->ctr, N, std::numeric_limits<int64_t>::max(), s->stream)))
        return done(hfail(s, e, "state restore"));
    e = hipStreamSynchronize(s->stream);
    if (e) return done(hfail(s, e, "backward"));
    return done(PSTD_OK);
}

}  // extern "C"
