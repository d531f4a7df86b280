// Internal interface between the host API and the device passes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pstd {

// Per-axis constant tables (device pointers), built in FP64 on the host and
// rounded once.
struct AxisTables {
    const float* kk;     // 2 eta dtau kbar_m^2 / N  (FFT index order)
    const float2* tw;    // exp(-2 pi i j / N), j = 0..N-1
    const float* gam;    // exp(-gamma(d) dtau), Eq. Gamma factor
    const float2* zt;    // zeta(i) exp(i khat_a x_a(i))
    const float2* dz;    // (zeta''(i) + 2 i khat_a zeta'(i)) exp(i khat_a x_a(i))
    const float4* zd;    // zt and dz of index i side by side: one 16-byte load per cell
    const float2* dlo;   // spectral-derivative row for the low plane
    const float2* dhi;   // spectral-derivative row for the high plane
};

// The potential term's factor 2 dtau (V / E0 + sum_a w_a) of Eq. PSTDupdating.
// V may be non-zero only where the taper is one (Section 2.2.2: (zeta - 1) V
// = 0), the box y1 <= i <= y2 of every axis, so it is stored on that box
// alone; w_a, the real part of a complex absorbing potential along axis a,
// is separable and comes from one table per axis (all null without it).
struct PotentialArgs {
    const float* box;      // 2 dtau V / E0 on the box, [z][y][x], x fastest
    int lo[3];             // first grid index of the box per axis
    int n[3];              // extent of the box per axis
    const float* wr[3];    // 2 dtau w_a(i) per grid index, or null
};

// Everything a pass launch needs for one solver instance and one axis.  The
// structs live in device memory and stay fixed while the solver runs; the
// per-step quantities are read on the device from the step counter:
// psi^n = buf[n & 1], psi^{n-1} = buf[(n + 1) & 1], and the tables below.
struct PassArgs {
    float2* buf[2];            // psi ping-pong
    float2* L;                 // kinetic accumulator (scaled by 2 eta dtau)
    PotentialArgs pot;
    int potx;                  // 1: the x pass takes the potential term (V's box covers few rows,
                               // no absorber real part, x unsegmented), else the z pass
    int nt;                    // 1: the fields outgrow the Infinity Cache; the z pass reads its
                               // last-use operands (psi^n, L, psi^{n-1}) with non-temporal loads
    int nx, ny, nz;
    AxisTables ax[3];
    const int64_t* ctr;        // device counters: ctr[0] = step n, ctr[1] = end (n >= end: no work)
    const float2* sigma_tab;   // per step: 2 dtau R(tau_n) exp(-i tau_n) [* eta]
    const double2* w_tab;      // per step: exp(i W tau_n), W the incident frequency
    const int* dft_tab;        // per step: 1 inside the surface-DFT window
    int plane_lo, plane_hi;    // plane indices along this pass's axis (local in segmented mode)
    double2* acc;              // [2 sides][4: sum psi, comp psi, sum dpsi, comp dpsi][points]
    float2* bstage;            // null, or (pulsed runs) [group step][2 sides][psi, dpsi][points]: the
                               // plane values are staged there instead of added to acc
    int64_t points;            // points of one plane of this axis
    // overlapping-subdomain mode along this pass's axis (Section 2.6)
    int seg_core, seg_halo, nseg;
    const float* wloc;         // local halo weights, length core + 2 halo
    int seg_plane[2];          // segment holding the low / high plane
    int tiles;                 // workgroups of this instance in this pass
    int ntx;                   // x tiles of the y and z passes
    // adjoint steps only: injected surface terms of this axis's low / high
    // planes (psi part, derivative part), the forward state each step pairs
    // with, and the gradient accumulator
    const float2* inj_lo_p;
    const float2* inj_lo_d;
    const float2* inj_hi_p;
    const float2* inj_hi_d;
    const float2* const* fwd_tab;
    float* grad;
    // forward steps only, may be null: per step, where to store a copy of
    // psi^{n+1} (null entry: no copy)
    float2* const* stash_tab;
};

// One FDTD-variant step (eighth-order stencil, Section 2.2.1) for one solver:
// psi^{n+1} = Gamma (psi^{n-1} - i q), q = kc psi + sum_a sum_l k[a][l-1]
// (psi(-l e_a) + psi(+l e_a)) + v2 psi + sigma_n sum_a dz_a prod_{b != a} zt_b
struct FdtdArgs {
    float2* buf[2];
    const float* v2;           // 2 dtau (V / E0 + sum_a w_a) on every cell (the stencil step reads it
                               // beside psi^{n-1}, at the same address)
    int nx, ny, nz;
    const float* gam[3];       // mask factors per axis
    const float2* zt[3];       // T_a e^{i kh_a x_a}
    const float2* dz[3];       // wall terms per axis (see fdtd.hip)
    const int64_t* ctr;
    const float2* sigma_tab;   // per step: 2 dtau R(tau_n) e^{-i tau_n}
    float kc;                  // -2 dtau alpha_0 sum_a 1 / dxb_a^2
    float k[3][4];             // -2 dtau alpha_l / dxb_a^2, l = 1..4
};
hipError_t launch_fdtd(const FdtdArgs& args, int koff, hipStream_t stream);
// the stencil coefficients of Eq. stencil_alpha
extern const double kFdtdAlpha[5];

// FFT-length configuration of a pass: N = N1 * N2, P pencils per workgroup;
// M1 > 0: stage B split as N2 = M1 * (N2 / M1) over all N2 threads of a pencil
struct PassShape {
    int N, N1, N2, P, threads, M1;
};

// Compiled tile-shape variants for local length N (segmented: with a
// subdomain instance).  Writes up to cap variant ids, returns the count.
int pass_variants(int N, bool segmented, int* out, int cap);
PassShape variant_shape(int v);
// Workgroups of variant v for one instance's pass along `axis`; also sets
// args.tiles and args.ntx.
int variant_tiles(int v, int axis, PassArgs& args);
// Launch variant v over a group of instances: descs[0..ninst) in device
// memory, off[0..ninst] (device) = prefix sums of their tiles.  The launch
// works on step ctr[0] + koff of each instance.
// The group's members all take the potential term where `potx` says (their
// PassArgs::potx); nt selects the z pass's non-temporal loads (PassArgs::nt).
hipError_t launch_variant(int v, bool segmented, int axis, const PassArgs* descs, const int* off, int ninst,
                          int total_tiles, int koff, int potx, int nt, hipStream_t stream);
// Bytes of the memory-side Infinity Cache of one MI355X; fields larger than
// this run their z passes with non-temporal loads.
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;
// Launch variant v for one instance described by `args` (passed by value)
hipError_t launch_variant_single(int v, bool segmented, int axis, const PassArgs& args, int koff, hipStream_t stream);
// Adjoint step pass (plain pencils, one instance)
hipError_t launch_variant_adjoint(int v, int axis, const PassArgs& args, int koff, hipStream_t stream);
// acc64[i] += acc32[i]; acc32[i] = 0
hipError_t launch_fold(double* acc64, float* acc32, int64_t n, hipStream_t stream);
// scratch[0] = sum |psi[i]|^2 (FP64) over n cells; scratch holds
// norm_scratch_doubles() doubles
int norm_scratch_doubles();
hipError_t launch_norm(const float2* psi, int64_t n, double* scratch, hipStream_t stream);
// out[i] = (float)(scale * acc64[i])
hipError_t launch_scale_out(const double* acc64, double scale, float* out, int64_t n, hipStream_t stream);
// advance the step counters of count instances by `by` steps, never past
// their end (ctr[2i] = step, ctr[2i+1] = end)
hipError_t launch_advance(int64_t* ctr, int count, int by, hipStream_t stream);

}  // namespace pstd
