// Near-to-distant-field projection (Section 3.2) on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/pstd.h"

namespace pstd {

struct ProjectState;  // cached spectra and expansion tables

// factors of the finalised phasors: values and normal derivatives (one over
// the incident phasor; the derivatives of a pulsed run's wavenumber k, taken
// in units rescaled by k, also over k)
struct PhasorScale {
    double2 v, d;
};
inline PhasorScale real_scale(double s) { return PhasorScale{make_double2(s, 0.0), make_double2(s, 0.0)}; }

// out[face][psi|dpsi][plane] = (sum + comp) * scale  (complex128)
hipError_t finalize_phasors(double2* const acc[3], const int64_t points[3], PhasorScale scale, double2* out,
                            hipStream_t stream);

hipError_t project_points(ProjectState** st, const pstd_problem& p, const double dxb[3], double2* const acc[3],
                          const int64_t points[3], PhasorScale scale, const double3* obs, int64_t n_obs, double2* out,
                          hipStream_t stream, std::string* msg);

hipError_t far_field(ProjectState** st, const pstd_problem& p, const double dxb[3], double2* const acc[3],
                     const int64_t points[3], PhasorScale scale, const double3* dirs, int64_t n_dir, double2* out,
                     hipStream_t stream, std::string* msg);

// Adjoint of project_points on the normalised phasors: given g (complex128,
// one per point), writes conj(G^H g) * scale as complex64 in the phasor
// layout (per face: psi plane, dpsi plane).
hipError_t project_adjoint(ProjectState** st, const pstd_problem& p, const double dxb[3], double2* const acc[3],
                           const int64_t points[3], double scale, const double3* obs, int64_t n_obs, const double2* g,
                           float2* inj, hipStream_t stream, std::string* msg);

void project_free(ProjectState* st);

}  // namespace pstd
