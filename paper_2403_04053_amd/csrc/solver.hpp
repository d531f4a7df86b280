// Solver state shared by the single-solver and batch entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pstd.h"
#include "internal.hpp"
#include "project.hpp"

namespace pstd {
struct AdjointState;  // misfit checkpoints and adjoint buffers
struct SphereState;   // spherical equivalence surface
struct PulseState;    // pulsed incidence
}

struct pstd_solver {
    pstd_problem prob{};
    hipStream_t stream = nullptr;
    int device = 0;
    double E0 = 0, dtau = 0, eta = 0, tau_r = 0;
    double omega = 1;      // frequency of the incident wave per unit tau (FDTD: the discrete one)
    double dxb[3] = {0, 0, 0};
    double kh[3] = {0, 0, 0};
    int64_t cells = 0;
    int64_t step = 0;      // host mirror of the device step counter
    double inc_sum = 0;    // incident phasor at the origin over the window steps run so far
    int64_t win_steps = 0; // window steps run so far
    float2* buf[2] = {nullptr, nullptr};
    float2* L = nullptr;
    float* vbox = nullptr;       // 2 dtau V / E0 on the taper's core
    float* wr = nullptr;         // complex absorber: 2 dtau w_a per axis (null without it)
    pstd::PotentialArgs pot{};
    float* v2full = nullptr;     // FDTD scheme only: 2 dtau (V / E0 + sum_a w_a) on every cell
    int potx = 0;                // the x pass takes the potential term (see solver_create)
    int nt = 0;                  // non-temporal loads in the z pass (see solver_create)
    void* tables = nullptr;
    pstd::AxisTables ax[3]{};
    const float* wloc[3] = {nullptr, nullptr, nullptr};
    double2* acc[3] = {nullptr, nullptr, nullptr};
    int64_t points[3] = {0, 0, 0};
    int variant[3] = {0, 0, 0};   // tile shape of each axis pass
    // per-step tables, steps [0, tab_cap)
    float2* sigma_tab = nullptr;
    double2* w_tab = nullptr;
    int* dft_tab = nullptr;
    int* dft_zero = nullptr;  // all zeros: the passes' box DFT is off with a spherical surface
    int64_t tab_cap = 0;
    int tab_gen = 0;       // bumped whenever the tables move
    // device counters (step, end); owned unless the solver belongs to a batch
    int64_t* ctr = nullptr;
    bool owns_ctr = true;
    // graph of kGraphSteps steps, replayed on `stream`
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    pstd::ProjectState* proj = nullptr;
    pstd::AdjointState* adj = nullptr;
    pstd::SphereState* sphere = nullptr;
    pstd::PulseState* pulse = nullptr;
    std::string err;
    bool in_batch = false;
};

namespace pstd {

pstd_status solver_create(const pstd_problem* p, hipStream_t stream, int64_t* ext_ctr, pstd_solver** out);
pstd_status solver_fail(pstd_solver* s, pstd_status st, const std::string& msg);
pstd_status solver_hip_fail(pstd_solver* s, hipError_t e, const char* what);
// make the per-step tables cover steps [0, n_end); refreshes the descriptors
pstd_status solver_ensure_tables(pstd_solver* s, int64_t n_end);
// fill the host copy of the descriptor of one axis
void solver_args(const pstd_solver* s, int axis, PassArgs& a);
// incident phasor bookkeeping for steps [from, to)
void solver_account_steps(pstd_solver* s, int64_t from, int64_t to);
pstd_status solver_autotune(pstd_solver* s, int32_t reps);
void solver_drop_graph(pstd_solver* s);
// the misfit forward run no longer matches the solver state
void adjoint_invalidate(pstd_solver* s);
void adjoint_free(pstd_solver* s);
// taper factor of axis a at index i with its first and second derivatives
// in the reduced coordinate (Eq. zeta_y)
void solver_taper(const pstd_problem& p, int a, double dxb, int i, double* z, double* z1, double* z2);
// zeta_a(i) exp(i khat_a xbar_i) for every grid index of axis a, FP64
void solver_incident_axis(const pstd_solver* s, int a, std::vector<double2>& out);

// spherical equivalence surface (sphere.hip)
pstd_status sphere_create(pstd_solver* s);
void sphere_free(SphereState* sp);
// running DFT of psi^{ctr[0] + koff} on the shell cells (inside the window)
// shell DFT of the `count` (1 or 2) steps ending at ctr[0] + koff, launched
// before that step's passes
hipError_t sphere_launch_dft(const pstd_solver* s, int koff, int count, hipStream_t stream);
hipError_t sphere_clear(pstd_solver* s, hipStream_t stream);
int64_t sphere_state_bytes(const pstd_solver* s);
hipError_t sphere_save(const pstd_solver* s, char* dst, hipStream_t stream);
hipError_t sphere_load(pstd_solver* s, const char* src, hipStream_t stream);
int64_t sphere_nodes(const pstd_solver* s);
// which phasor set an output reads: wavenumber index, the factor that
// normalises it (one over the incident phasor) and the reduced wavenumber
struct SphereOut {
    int ik;
    double2 scale;
    double k;
};
// node phasors (psi, d_n psi; scattered part, normalised)
hipError_t sphere_phasors(pstd_solver* s, const SphereOut& o, double2* out, hipStream_t stream);
hipError_t sphere_project(pstd_solver* s, const SphereOut& o, const double3* obs, int64_t n_obs, double2* out,
                          hipStream_t stream);
hipError_t sphere_far_field(pstd_solver* s, const SphereOut& o, const double3* dirs, int64_t n_dir, double2* out,
                            hipStream_t stream);
// phasor sums for nk wavenumbers (cleared) and the ring of staged steps:
// a pulsed run stages psi on the shell each step and adds a launch group's
// steps to the sums once, at its end
constexpr int kStageSteps = 16;  // steps per launch group at most
hipError_t sphere_set_wavenumbers(pstd_solver* s, int nk);
bool sphere_staged(const pstd_solver* s);
void sphere_drop_stage(pstd_solver* s);
hipError_t sphere_launch_stage(const pstd_solver* s, int koff, hipStream_t stream);
hipError_t sphere_launch_flush(const pstd_solver* s, int count, hipStream_t stream);
// the shell list and the ring (null without staging) for a fused launch
void sphere_stage_buffers(const pstd_solver* s, const int** list, int64_t* n_shell, float2** stage);
// largest taper value on the shell cells
double sphere_taper_max(const pstd_solver* s);

// pulsed incidence (pulse.hip)
pstd_status pulse_set(pstd_solver* s, const double* psi0, int32_t n1d, double delta, const double* kbar, int32_t nk);
void pulse_free(PulseState* p);
int pulse_wavenumbers(const pstd_solver* s);
// a pulsed run's first step since the pulse was set or pstd_set_state
int64_t pulse_from(const pstd_solver* s);
double pulse_frequency(const pstd_solver* s, int ik);
// before the x pass of step ctr[0] + koff: the packet's table of the next
// step, the layer source of this one (added to psi^{n-1}), and psi^n of the
// shell cells `list` into slot koff of `stage` (when stage is not null);
// koff = -1 primes the table of step ctr[0]
hipError_t pulse_launch_pre(const pstd_solver* s, int koff, const int* list, int64_t n_shell, float2* stage,
                            hipStream_t stream);
// the steps that count for the incident phasors start at the current step
void pulse_reset(pstd_solver* s);
// checkpoint of a pulsed run: the box's per-wavenumber plane sums (the
// sphere's are saved with the sphere); pulse_load also restores the first
// step since the last reset and primes the packet's table of the current
// step, so the device counter must already hold it
int64_t pulse_state_bytes(const pstd_solver* s);
hipError_t pulse_save(const pstd_solver* s, char* dst, hipStream_t stream);
hipError_t pulse_load(pstd_solver* s, const char* src, int64_t from);
// the output of wavenumber ik
pstd_status pulse_output(pstd_solver* s, int ik, SphereOut* o);
// box surface: the staging ring of the pass along `axis` (null unless a
// pulsed run integrates over the box), the group flush, and the inputs of the
// box projection for wavenumber ik (rescaled: units of that wavenumber)
float2* pulse_box_stage(const pstd_solver* s, int axis);
hipError_t pulse_launch_box_flush(const pstd_solver* s, int count, hipStream_t stream);
struct BoxOut {
    pstd_problem prob;
    double dxb[3];
    double2* acc[3];
    PhasorScale scale;
    ProjectState** proj;
};
pstd_status pulse_box_output(pstd_solver* s, int ik, bool rescaled, BoxOut* o);

}  // namespace pstd
