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
    const float2* dlo;   // spectral-derivative row for the low plane
    const float2* dhi;   // spectral-derivative row for the high plane
};

struct PassArgs {
    const float2* psi;   // psi^n
    float2* L;           // kinetic accumulator (scaled by 2 eta dtau)
    float2* psi_old;     // psi^{n-1} in, psi^{n+1} out (z pass)
    const float* v2;     // 2 dtau V / E0
    int nx, ny, nz;
    AxisTables ax[3];
    float2 sigma;        // 2 dtau R(tau_n) exp(-i tau_n) [* eta]
    int dft_on;
    double2 w;           // exp(i tau_n)
    int plane_lo, plane_hi;  // plane indices along this pass's axis
    double2* acc;        // [2 sides][4: sum psi, comp psi, sum dpsi, comp dpsi][points]
    int64_t points;      // points of one plane of this axis
    // overlapping-subdomain mode along this pass's axis (Section 2.6)
    int seg_core, seg_halo, nseg;
    const float* wloc;   // local halo weights, length core + 2 halo
    int seg_plane[2];    // segment holding the low / high plane (plane_lo/hi are local then)
};

// FFT-length configuration of a pass: N = N1 * N2, P pencils per workgroup
struct PassShape {
    int N, N1, N2, P, threads;
};

// Compiled tile-shape variants for local length N (segmented: with a
// subdomain instance).  Writes up to cap variant ids, returns the count.
int pass_variants(int N, bool segmented, int* out, int cap);
PassShape variant_shape(int v);
// Launch variant v for the pass along `axis` (0, 1, 2)
hipError_t launch_variant(int v, bool segmented, int axis, const PassArgs& args, hipStream_t stream);

}  // namespace pstd
