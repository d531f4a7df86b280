/*
 * libpstd — C ABI of the MI355X PSTD quantum-scattering hot path.
 *
 * The library advances the Schroedinger wave function of a scattering problem
 * on a 3D grid with the pseudo-spectral leapfrog of Eq. PSTDupdating
 * (Section 2.5 of Chen, arXiv 2403.04053): per-axis spectral kinetic term,
 * potential term, total-field/scattered-field plane-wave source (Section
 * 2.2.2), masking absorber (Section 2.1, Eq. Gamma).  During a time window it
 * accumulates the running DFT of psi and of its normal derivative on the six
 * faces of a virtual box (Section 3.3, Eqs. psiphasor, dpsiphasor), and
 * projects those phasors to distant points or to far-field directions with
 * the semi-analytic surface integral of Section 3.2 (Eqs. bottomPsi_lm ...
 * Psi).
 *
 * Conventions (every call):
 *  - grid index (i, j, k) along (x, y, z) is the physical point
 *    ((i - Nx/2) hx, (j - Ny/2) hy, (k - Nz/2) hz); 3D arrays are [k][j][i]
 *    (x fastest), n_cells = Nx*Ny*Nz;
 *  - complex64 = interleaved float (re, im); complex128 = interleaved double;
 *  - a pointer named *_dev is device memory on the device current when the
 *    solver was created; *_host is host memory.  The caller owns every pointer
 *    it passes; the library keeps none after the call returns;
 *  - every call that launches work enqueues it on the stream given at
 *    creation (0 = the null stream) and returns without synchronising, except
 *    where the description says it synchronises;
 *  - one solver is used by one host thread at a time; solvers are independent;
 *  - no call aborts: each returns a pstd_status, and pstd_last_error() gives
 *    a message for the last failing call on that solver.
 */
#ifndef PSTD_H
#define PSTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pstd_status {
    PSTD_OK = 0,
    PSTD_EINVAL = 1,       /* bad argument, size, index or geometry */
    PSTD_EUNSTABLE = 2,    /* dt above the bound of Eq. PSTDstability */
    PSTD_ENONFINITE = 3,   /* NaN/Inf in an input or in the wave function */
    PSTD_ENOMEM = 4,       /* device allocation failed */
    PSTD_EHIP = 5,         /* a HIP runtime call failed */
    PSTD_ESTATE = 6,       /* call not valid in the solver's current state */
    PSTD_EUNSUPPORTED = 7  /* grid length without a compiled FFT pass */
} pstd_status;

/*
 * Problem description (physical units unless stated).  Section 2 defines the
 * internal model: absorbing layer (Section 2.1), TF/SF taper (Eq. zeta_y),
 * plane-wave incidence of wavenumber k0 along the direction of Eq. khat,
 * virtual box (Section 3.1).
 */
typedef struct pstd_problem {
    int32_t n[3];            /* FFT grid points per axis; even */
    double  h[3];            /* grid spacing per axis */
    double  hbar, mass;      /* > 0 */
    double  k0;              /* central wavenumber of the incident wave, > 0 */
    double  theta, phi;      /* incident direction, Eq. khat (radians) */
    int32_t abc_cells[3];    /* absorbing-layer width per axis, cells */
    double  abc_U0;          /* Eq. Poshcl-Teller height, units of E0/hbar */
    double  abc_alpha;       /* Eq. Poshcl-Teller decay, per cell */
    int32_t tfsf[3][4];      /* y0 < y1 <= y2 < y3 per axis, Eq. zeta_y */
    double  v_max;           /* bound on |V| used for the step (energy) */
    double  dt;              /* time step; 0 selects 0.9 of the critical one */
    int32_t force_dt;        /* 1: accept dt above the bound */
    double  ramp_periods;    /* switch-on length of the incident wave */
    int64_t dft_begin;       /* surface-DFT window [dft_begin, dft_end) */
    int64_t dft_end;
    int32_t surf_lo[3];      /* box faces: grid indices per axis */
    int32_t surf_hi[3];
    int32_t eta_on_source;   /* 1: scale the source by eta as well */
    /* Overlapping subdomains with local Fourier basis (Section 2.6): along
     * every axis with sub_core[a] > 0 the kinetic term is taken on local
     * arrays of sub_core[a] + 2 sub_halo points (halo weighted by Eq. weight
     * with sub_taper tapered points) and only core points are updated.
     * n[a] must be a multiple of sub_core[a]; sub_halo >= sub_taper + 5. */
    int32_t sub_core[3];
    int32_t sub_halo;
    int32_t sub_taper;
    /* Equivalence surface used by pstd_project / pstd_far_field.  Section 3.1
     * allows any closed surface around the scatterer; the paper integrates
     * over the box faces (surface_kind 0).  surface_kind 1 uses a sphere of
     * radius sphere_radius (physical, centred at the origin) with
     * sphere_nodes = (n_theta, n_phi) Gauss-Legendre x uniform quadrature
     * nodes (0, 0: 64 x 128): the running DFT is taken on the shell of grid
     * cells that 8-point Lagrange stencils around the nodes touch, the
     * incident part zeta psi_inc is removed, and the Kirchhoff integral with
     * G = exp(ikR)/(4 pi R) is summed over the nodes; the box faces are then
     * not accumulated.  The sphere must enclose the region where the taper is
     * one and its shell must stay outside the absorber. */
    int32_t surface_kind;
    int32_t sphere_nodes[2];
    double  sphere_radius;
    /* Complex absorbing potential (Section 2.1: the absorbing potential may be
     * complex while its imaginary part stays non-positive).  The imaginary
     * part is the mask above; abc_UR (units of E0) adds the real part
     * w(d) = abc_UR / cosh^2(abc_alphaR d) inside the layer of every axis,
     * summed over the axes, to the potential of the step.  abc_alphaR = 0
     * takes abc_alpha.  The step bound then uses max(v_max / E0, |abc_UR|
     * times the number of axes with a layer).  0, 0: the mask alone. */
    double  abc_UR;
    double  abc_alphaR;
    /* Step scheme.  0: the spectral step of Eq. PSTDupdating.  1: the FDTD
     * variant of Section 2.2.1: the eighth-order central stencil of Eq.
     * y_stencil (Eq. stencil_alpha) on the periodic grid, Eq.
     * FDTDupdatePsi with V multiplying psi^n, no eta correction, a sharp
     * total-field box y1 <= i <= y2 per axis whose walls carry the
     * consistency terms of Eqs. FDTDpsi_extraJminus1-FDTDpsiJplus4 (y0, y3
     * unused), the same mask; step bound dtau <= 1 / (|alpha_0 + 2 sum_l
     * alpha_l (-1)^l| sum_a 1/dxb_a^2 + |v|max).  The walls drive the
     * incident wave at the scheme's discrete frequency W for k_hat,
     * sin(W dtau) = dtau k_h^2 (k_h^2 the stencil's symbol summed over the
     * axes), and the surface DFT weighs step n with exp(i W tau_n).  Scheme 1
     * takes the spherical surface (surface_kind 1) for the surface DFT and
     * the projection; a DFT window with the box surface, subdomains, batch
     * instances and the misfit return EUNSUPPORTED. */
    int32_t scheme;
} pstd_problem;

typedef struct pstd_solver pstd_solver;  /* opaque; owns all its device memory */

/* Fill *p with a small valid default problem.  Host only, no allocation. */
pstd_status pstd_problem_init_defaults(pstd_problem* p);

/* Critical step of Eq. PSTDstability for |V| <= vmax (energy units):
 * dt_c = hbar / (hbar^2 pi^2 / 2m * sum_a 1/h_a^2 + vmax).  Host only. */
pstd_status pstd_critical_dt(const pstd_problem* p, double vmax, double* dt_out_host);

/* Reduced step dtau = E0 dt / hbar and phase-velocity factor eta =
 * sin(dtau)/dtau (Eq. numdis2) the solver uses.  Host only. */
pstd_status pstd_reduced_step(const pstd_problem* p, double* dtau_out_host, double* eta_out_host);

/* Validate p, allocate the solver's device state on the current device and
 * build its tables (FP64 on the host, rounded once; the per-step tables
 * cover max(1024, dft_end) steps, at most 2^18, and grow when a run goes
 * further).  psi^{-1} = psi^0 = 0, V = 0, step index 0.  hip_stream: a
 * hipStream_t or 0.  Synchronises.
 * EINVAL: odd or tiny n, taper indices out of order, a box face that is not
 * wholly in the scattered-field region (zeta = 0 on the whole plane) or
 * inside the absorber.  EUNSTABLE: dt above the bound and force_dt = 0.
 * EUNSUPPORTED: an axis length (or local subdomain length) with no compiled
 * FFT pass. */
pstd_status pstd_create(const pstd_problem* p, void* hip_stream, pstd_solver** out);

/* Copy the potential V (float32, energy units, [k][j][i]) into the solver as
 * 2 dtau V / E0.  Synchronises.  EINVAL: n_cells mismatch.  ENONFINITE: a
 * NaN/Inf value.  EUNSTABLE: max|V| > v_max (the step was sized for v_max).
 * EINVAL also when V != 0 where the taper is below one ((zeta - 1) V = 0,
 * Section 2.2.2). */
pstd_status pstd_set_potential(pstd_solver* s, const float* V_dev, int64_t n_cells);

/* Replace (psi^{n-1}, psi^n) by two complex64 device arrays and set the step
 * index to `step` (the next step computes psi^{step+1}).  Clears the surface
 * DFT.  For restarts and tests. */
pstd_status pstd_set_state(pstd_solver* s, const void* psi_prev_dev, const void* psi_cur_dev,
                           int64_t n_cells, int64_t step);

/* Advance n_steps leapfrog steps of Eq. PSTDupdating; accumulate the surface
 * DFT for the steps inside [dft_begin, dft_end).  Asynchronous. */
pstd_status pstd_run(pstd_solver* s, int64_t n_steps);

/* Like pstd_run (without the graph), and also times every pass kernel with
 * a pair of HIP events around its launch on the solver's stream; the steps
 * are queued back to back and the events read at the end.  pass_ms_host[3]
 * receives the summed milliseconds of the x, y and z passes.  Synchronises. */
pstd_status pstd_run_timed(pstd_solver* s, int64_t n_steps, double* pass_ms_host);

/* Pick, for each axis pass, the fastest compiled tile shape (FFT factor
 * order N1 x N2 and pencils per workgroup) by timing `reps` launches of every
 * candidate on scratch buffers of the solver's size, in two rounds (each
 * candidate keeps the faster of its two timings); the solver's state is
 * not touched.  Candidates are compared in compiled order and a later one
 * replaces the current choice only when it is at least 3 % faster, so timing
 * noise does not flip the choice between runs.  Also captures the step graph
 * of the chosen shapes, so that the next pstd_run does not.  Synchronises.
 * ENOMEM if the scratch cannot be allocated. */
pstd_status pstd_autotune(pstd_solver* s, int32_t reps);

/* Failure detection: *norm2_out_host = sum over the cells of |psi^step|^2
 * (FP64; compare it between calls to watch for growth).  ENONFINITE if
 * psi^step or psi^{step-1} holds a NaN or Inf (e.g. a step forced above the
 * bound of Eq. PSTDstability with force_dt).  Synchronises. */
pstd_status pstd_check_state(pstd_solver* s, double* norm2_out_host);

/* pstd_check_state for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same result, errors
 * and synchronisation, with the reduction's partial sums in a fixed device
 * array of 4096 doubles (32 KiB) per device, which the library holds until
 * the process ends, instead of a buffer allocated and freed per call.  Calls
 * no hipMalloc, hipFree or other allocating routine (the array's address on
 * each device is looked up once, by pstd_create on that device).  Calls on
 * one device share its array: the library serialises them with a lock held
 * until the result is read (overlapping uses of one device's array would
 * race).  EINVAL if the reduction needed more than the array holds. */
pstd_status pstd_check_state_noalloc(pstd_solver* s, double* norm2_out_host);

/* Average duration (microseconds) of one launch of the pass along `axis`
 * with its current tile shape: `reps` back-to-back launches on scratch
 * buffers of the solver's size, bracketed by HIP events on the solver's
 * stream (the same timing the autotuner uses).  The solver's state is not
 * touched.  Synchronises. */
pstd_status pstd_pass_time(pstd_solver* s, int32_t axis, int32_t reps, double* us_out_host);

/* Tile shape used by the pass along axis (0, 1, 2): info_host[5] =
 * {N, N1, N2, pencils per workgroup, M1}; M1 > 0 when stage B (the N2-point
 * DFTs) is split as N2 = M1 * (N2 / M1) over all N2 threads of a pencil, 0
 * otherwise.  Host only. */
pstd_status pstd_tile_info(const pstd_solver* s, int32_t axis, int32_t* info_host);

/* Use the compiled tile shape of axis `axis` with stage-A factor n1,
 * `pencils` pencils per workgroup and stage-B split m1 (0: none).
 * EUNSUPPORTED if there is none.  Synchronises. */
pstd_status pstd_set_tile(pstd_solver* s, int32_t axis, int32_t n1, int32_t pencils, int32_t m1);

/* Compiled tile shapes for pass length n (segmented != 0: subdomain mode):
 * writes up to cap quadruples {N1, N2, pencils, M1} to shapes_host[4*cap]
 * and the total number to *count_out.  Host only. */
pstd_status pstd_tile_variants(int32_t n, int32_t segmented, int32_t* shapes_host, int32_t cap, int32_t* count_out);

/* Number of steps taken (the current level is psi^step). */
pstd_status pstd_step_index(const pstd_solver* s, int64_t* step_out_host);

/* Copy psi^step (level 0) or psi^{step-1} (level 1) to a complex64 array. */
pstd_status pstd_get_psi(pstd_solver* s, int32_t level, void* psi_dev, int64_t n_cells);

/* Checkpoint / resume of a solve: pstd_state_size gives the bytes of a
 * device buffer that holds (psi^{n-1}, psi^n), the FP64 surface-DFT sums with
 * their compensation terms, the step index and the incident-phasor sum.
 * pstd_save_state fills such a buffer (caller-owned device memory);
 * pstd_load_state restores it into a solver of the same grid, after which
 * pstd_run continues exactly as the saved solver would (bit-identical
 * results).  A pulsed run's state adds its first step and the sums of every
 * wavenumber; load it into a solver given the same pulse (pstd_set_pulse
 * with the same packet and wavenumbers, before the load).  Both synchronise.
 * EINVAL: buffer too small, or (load) a buffer that holds no state of this
 * grid, or whose run differs from this solver in having a pulse or in its
 * number of wavenumbers.  ESTATE: load into a batch instance. */
pstd_status pstd_state_size(const pstd_solver* s, int64_t* bytes_out_host);
pstd_status pstd_save_state(pstd_solver* s, void* dev_buf, int64_t bytes);
pstd_status pstd_load_state(pstd_solver* s, const void* dev_buf, int64_t bytes);

/* Number of complex128 values pstd_get_surface_phasors writes:
 * 2 * (2 Ny Nz + 2 Nx Nz + 2 Nx Ny). */
pstd_status pstd_surface_size(const pstd_solver* s, int64_t* n_out_host);

/* Normalised phasors of Eqs. scaledphsiphasor / scaleddpsiphasor, divided by
 * the incident phasor at the coordinate origin (the switch-on ramp summed
 * over the window steps that have run since creation or pstd_set_state).  Layout: faces x-lo, x-hi, y-lo, y-hi, z-lo, z-hi; per
 * face the psi plane then the d(psi)/d(x_bar_normal) plane (reduced-unit
 * derivative); x faces are [k][j], y faces [k][i], z faces [j][i].
 * ESTATE if no step of the window has run, or with a spherical surface. */
pstd_status pstd_get_surface_phasors(pstd_solver* s, double* out_dev, int64_t n);

/* Number of quadrature nodes of the spherical surface (0 for the box). */
pstd_status pstd_sphere_size(const pstd_solver* s, int64_t* n_nodes_out_host);

/* Scattered-field phasors at the sphere's nodes, normalised like the box
 * phasors: out_dev = [psi at the nodes][d psi / d n_bar at the nodes],
 * complex128, n = 2 * pstd_sphere_size; nodes ordered [theta][phi] with
 * cos(theta) ascending (Gauss-Legendre) and phi = 2 pi j / n_phi.  ESTATE
 * without a sphere or before any window step. */
pstd_status pstd_get_sphere_phasors(pstd_solver* s, double* out_dev, int64_t n);

/* Scattered wave Psi(r) at n_obs points (physical xyz, double[3] each) by the
 * box integral of Eqs. bottomPsi_lm ... leftrightPsi_ln summed by Eq. Psi,
 * with each sinc expanded to 8th order in its shift.  Output complex128,
 * relative to a unit-amplitude incident wave.  Points must lie outside the
 * box (outside the sphere with surface_kind 1, which sums the Kirchhoff
 * integral over the sphere's nodes instead).  ESTATE before any window
 * step.  n_obs = 0 does nothing and returns PSTD_OK (the pointers may then
 * be null). */
pstd_status pstd_project(pstd_solver* s, const double* obs_xyz_dev, int64_t n_obs, double* psi_out_dev);

/* Far-field amplitude f(r_hat) = lim r e^{-ikr} Psi (physical length units)
 * for n_dir unit directions (double[3] each): the cell formula in the limit
 * of Eq. FDTDfarfieldapprox (with surface_kind 1, the limit of the sphere's
 * Kirchhoff sum).  Output complex128.  n_dir = 0 does nothing and returns
 * PSTD_OK (the pointers may then be null). */
pstd_status pstd_far_field(pstd_solver* s, const double* dir_dev, int64_t n_dir, double* f_out_dev);

/*
 * Pulsed (broadband) incidence: Section 2.2.3, calculation of the incident
 * wave (Eqs. Oinc, inc_d, pstd_psiinc, pstd_dpsiinc), and Section 3.3 with
 * several frequencies (Eqs. psiphasor-scaleddpsiphasor repeated per
 * frequency).
 *
 * Replaces the monochromatic plane wave of the solve by a packet of any
 * shape travelling along k_hat.  psi0_host: the packet at step 0 on the
 * periodic 1D grid d_j = j delta (reduced length, d = 0 at the corner of
 * the taper box that the front reaches first, Eq. Oinc; a cell sits at d =
 * k_hat . (x - x_O), Eq. inc_d), n1d complex values as interleaved FP64
 * (re, im) in host memory, copied.  The packet advances by the leapfrog of
 * Eq. PSTDupdating in 1D (free space, eta on the kinetic term), started on
 * each mode's physical root so that it travels one way; each step its value
 * and gradient at the transition-layer cells come from Eqs. pstd_psiinc and
 * pstd_dpsiinc (the spectral sum evaluated on a table four times finer than
 * the grids and interpolated from it with 8-point Lagrange weights: within
 * 1e-8 of the packet), and the layer source of Eq. dimlesstildeSchrodinger
 * is added to the step; the monochromatic source is off.  The 1D grid must
 * be long enough that the packet does not come round again during the run.
 *
 * kbar_host: n_k reduced wavenumbers k/k0 (host, copied).  The spherical
 * surface accumulates one phasor per wavenumber over the DFT window, step n
 * weighted by exp(i W tau_n) with sin(W dtau) = dtau eta kbar^2 (the
 * scheme's frequency of that wavenumber), each normalised by the incident
 * phasor at the grid origin (the DFT of the packet there over the same
 * steps); the _k outputs below project it with G = exp(i kbar R)/(4 pi R).
 *
 * With the box surface (surface_kind 0) the passes stage the plane values of
 * each launch group of steps and one flush per group adds them to a set of
 * plane sums per wavenumber; the box projection of wavenumber k is the
 * central wave's in units rescaled by k (k0 -> k k0, dxb -> k dxb).
 *
 * Requires the spectral scheme, an equivalence surface where the taper is
 * zero (box planes at or outside the taper box; or the sphere's
 * interpolation shell), no subdomains and no batch (EUNSUPPORTED
 * otherwise; the misfit refuses a pulsed solver); call before the first
 * step (ESTATE).
 * EINVAL: n1d not a power of two in [8, 2^20], delta <= 0, n_k outside
 * [1, 64], a wavenumber <= 0 or beyond the step bound, the 1D grid's
 * Nyquist mode beyond the step bound, a non-finite or zero packet, a
 * spectrum so wide that the layer's table would exceed 2^26 entries.
 * Synchronises. */
pstd_status pstd_set_pulse(pstd_solver* s, const double* psi0_host, int32_t n1d, double delta,
                           const double* kbar_host, int32_t n_k);

/* pstd_get_surface_phasors, pstd_get_sphere_phasors, pstd_project and
 * pstd_far_field for the phasors of wavenumber index ik of a pulsed run (the
 * plain calls read index 0; without a pulse ik must be 0).  The box
 * phasors' derivatives are per reduced length of the grid, as for the
 * central wave.  EINVAL for an index out of range. */
pstd_status pstd_get_surface_phasors_k(pstd_solver* s, int32_t ik, double* out_dev, int64_t n);
pstd_status pstd_get_sphere_phasors_k(pstd_solver* s, int32_t ik, double* out_dev, int64_t n);
pstd_status pstd_project_k(pstd_solver* s, int32_t ik, const double* obs_xyz_dev, int64_t n_obs,
                           double* psi_out_dev);
pstd_status pstd_far_field_k(pstd_solver* s, int32_t ik, const double* dir_dev, int64_t n_dir,
                             double* f_out_dev);

/*
 * Differentiation with respect to the voxel potential (not in the paper; the
 * discrete adjoint of Eq. PSTDupdating, of the surface DFT of Eqs. psiphasor /
 * dpsiphasor / scaledphsiphasor and of the box projection of Section 3.2).
 *
 * Misfit of a detector-plane intensity:
 *   J(V) = 1/2 sum_o (|exp(i k0 khat . r_o) + Psi_o|^2 - I_o)^2,
 * Psi_o = pstd_project at the points r_o, I_o the target intensities.
 */

/* From rest (psi^{-1} = psi^0 = 0, step 0, surface DFT cleared), run n_steps
 * steps with the current potential, keeping n_checkpoints checkpoint pairs
 * (psi^{kS-1}, psi^{kS}) at the segment starts kS, S = ceil(n_steps /
 * n_checkpoints), and evaluate J (written to *J_out_host, FP64).
 * obs_xyz_dev: n_obs physical points (double[3] each, outside the box);
 * target_I_dev: n_obs doubles.  Both are copied.  Device memory held until
 * pstd_destroy or a forward call with other sizes:
 * (2 n_checkpoints + S + 5) complex64 fields of the grid plus one FP64 field.
 * Synchronises.  EINVAL: n_checkpoints outside [1, n_steps], no window step
 * before n_steps, a point inside the box.  EUNSUPPORTED: segmented axes.
 * ESTATE: a batch instance.  ENONFINITE: J is not finite. */
pstd_status pstd_misfit_forward(pstd_solver* s, int64_t n_steps, const double* obs_xyz_dev, int64_t n_obs,
                                const double* target_I_dev, int32_t n_checkpoints, double* J_out_host);

/* dJ/dV (float32, energy^-1 per cell times energy^2 of J: d J / d V_c in the
 * units of V, layout [k][j][i]) of the last pstd_misfit_forward.  Recomputes
 * each segment from its checkpoint and runs the adjoint steps backwards
 * (about two forward steps of work per step).  The gradient covers every
 * cell; pstd_set_potential accepts V only where the taper is one, so callers
 * mask the rest.  Leaves the solver in the state the forward run ended in and
 * may be called again.  Synchronises.  ESTATE: no forward run, or the solver
 * stepped, took a new potential or state since. */
pstd_status pstd_misfit_backward(pstd_solver* s, float* dJdV_dev, int64_t n_cells);

pstd_status pstd_destroy(pstd_solver* s);

/*
 * Batched solves.  `count` independent problems (own grids, directions,
 * energies, potentials, steps) advanced together: per axis the instances are
 * grouped by FFT tile shape and each group is one launch; step groups are
 * replayed from a HIP graph.  Every instance has the single-solver state and
 * tables.
 */
typedef struct pstd_batch pstd_batch;  /* opaque; owns its instances */

/* Create `count` instances from problems[0..count) on the current device.
 * Synchronises.  Errors as pstd_create; the message names the instance. */
pstd_status pstd_batch_create(const pstd_problem* problems, int32_t count, void* hip_stream, pstd_batch** out);
pstd_status pstd_batch_size(const pstd_batch* b, int32_t* count_out_host);
/* Borrowed handle of instance idx, for pstd_get_psi, pstd_get_surface_phasors,
 * pstd_project, pstd_far_field, pstd_step_index, pstd_tile_info.  Owned by
 * the batch: never pass it to pstd_destroy; pstd_run on it returns ESTATE
 * (pstd_set_state works and takes effect at the next pstd_batch_run). */
pstd_status pstd_batch_solver(pstd_batch* b, int32_t idx, pstd_solver** out);
/* pstd_set_potential for instance idx. */
pstd_status pstd_batch_set_potential(pstd_batch* b, int32_t idx, const float* V_dev, int64_t n_cells);
/* Tile autotuning: the largest instance of each distinct pass length is
 * tuned (as pstd_autotune) and its choice shared.  Synchronises. */
pstd_status pstd_batch_autotune(pstd_batch* b, int32_t reps);
/* Advance instance i by n_steps_host[i] steps (0 allowed); instances that
 * reach their count stop while the others continue.  Asynchronous after the
 * counters are set. */
pstd_status pstd_batch_run(pstd_batch* b, const int64_t* n_steps_host);
pstd_status pstd_batch_destroy(pstd_batch* b);
const char* pstd_batch_last_error(const pstd_batch* b);

const char* pstd_status_string(pstd_status st);
const char* pstd_last_error(const pstd_solver* s);

#ifdef __cplusplus
}
#endif

#endif /* PSTD_H */
