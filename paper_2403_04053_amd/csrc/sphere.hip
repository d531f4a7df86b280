// Spherical equivalence surface (Section 3.1 allows any closed surface; the
// paper integrates over a box).  Nodes: Gauss-Legendre in cos(theta) times
// uniform phi on a sphere centred at the origin.  Every window step
// accumulates, in FP64, the DFT of psi (Eq. psiphasor) on the shell of grid
// cells that the 8-point Lagrange stencils around the nodes touch.  After
// the run the node values and normal derivatives come from the separable
// Lagrange interpolant of the scattered-field phasors (the incident
// part zeta exp(i khat . x) is removed exactly), and the Kirchhoff integral
// with G = exp(ikR)/(4 pi R) is summed over the nodes, in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "solver.hpp"

namespace pstd {

constexpr int kStencil = 8;

struct SphereState {
    int n_nodes = 0;
    double R = 0;                 // reduced radius
    double3* node = nullptr;      // reduced coordinates
    double3* normal = nullptr;
    double* weight = nullptr;
    int* start = nullptr;         // [node][3] stencil start per axis
    double* lw = nullptr;         // [node][3][2][kStencil]: weights, derivative weights (per reduced length)
    int64_t n_shell = 0;
    int* list = nullptr;          // shell cells (linear index), ascending
    int* slot = nullptr;          // grid -> shell slot (-1 outside)
    double2* inc = nullptr;       // zeta exp(i khat . x) per shell slot
    double inc_max = 0;           // largest |zeta| on the shell (0: scattered field only)
    int nk = 1;                   // wavenumbers with a phasor (more than one with a pulse)
    double2* sum = nullptr;       // running DFT [wavenumber][slot]
    double2* comp = nullptr;      // same layout, all zero: the kernels keep plain FP64 sums (the node
                                  // interpolation adds it, the saved state carries it)
    float2* stage = nullptr;      // [kStageSteps][slot]: psi of the steps of a launch group (pulsed runs)
    double2* phasor = nullptr;    // [2][node]: psi, d_n psi
};

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// n-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1);
            const double d = p1 / dp;
            t -= d;
            if (std::fabs(d) < 1e-16) break;
        }
        double p0 = 1, p1 = t;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1);
        x[n - 1 - i] = t;  // ascending
        w[n - 1 - i] = 2.0 / ((1 - t * t) * dp * dp);
    }
}

// stencil start and Lagrange weights (and derivative weights per unit index)
// of kStencil points at fractional index u
int lagrange(double u, double* L, double* dL) {
    const int i0 = (int)std::floor(u) - (kStencil / 2 - 1);
    for (int m = 0; m < kStencil; ++m) {
        double den = 1, num = 1, der = 0;
        for (int j = 0; j < kStencil; ++j) {
            if (j == m) continue;
            den *= (double)(m - j);
            // d/du of prod_j (u - x_j): sum over the dropped factor
            der = der * (u - (i0 + j)) + num;
            num *= (u - (i0 + j));
        }
        L[m] = num / den;
        dL[m] = der / den;
    }
    return i0;
}

// Eq. psiphasor on the shell cells for `count` (1 or 2) consecutive steps
// ending at ctr[0] + koff, each with its own weight and window flag.  Run
// before that step's z pass, when both psi^{n-1} and psi^n are in place, so
// a pair of steps costs one read-modify-write of the FP64 sums; the terms
// are added in step order, as one launch per step would.  One wavenumber
// (a pulsed run's several go through the staged path below).
// Plain FP64 sums: each term is an FP32 value times a unit phase, and W
// additions in FP64 err by at most about W 2^-53 of the sum of the terms'
// moduli (under 2e-12 for the 14 440 steps of the longest run), far below the
// 2^-24 of the field itself; the compensation array, which the node
// interpolation adds to the sums, stays zero on this path (52 B per cell
// and pair of steps instead of 84).
__global__ void shell_dft_kernel(const int64_t* __restrict__ ctr, int koff, int count, const int* __restrict__ dft_tab,
                                 const double2* __restrict__ w_tab, const float2* __restrict__ buf0,
                                 const float2* __restrict__ buf1, const int* __restrict__ list, int64_t n,
                                 double2* __restrict__ sum) {
    const int64_t last = ctr[0] + koff;
    const int64_t first = last - (count - 1);
    bool any = false;
    for (int64_t m = first; m <= last; ++m) any |= m < ctr[1] && dft_tab[m] != 0;
    if (!any) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int cell = list[c];
    double2 s = sum[c];
    for (int64_t m = first; m <= last; ++m) {
        if (m >= ctr[1] || !dft_tab[m]) continue;
        const float2 x = ((m & 1) ? buf1 : buf0)[cell];
        const double2 w = w_tab[m];
        s.x += w.x * x.x - w.y * x.y;
        s.y += w.x * x.y + w.y * x.x;
    }
    sum[c] = s;
}

// psi^n on the shell cells into slot koff of the ring, n = ctr[0] + koff,
// before step n's passes (psi^n is in place until step n + 1)
__global__ void shell_stage_kernel(const int64_t* __restrict__ ctr, int koff, const float2* __restrict__ buf0,
                                   const float2* __restrict__ buf1, const int* __restrict__ list, int64_t n,
                                   float2* __restrict__ stage) {
    const int64_t m = ctr[0] + koff;
    if (m >= ctr[1]) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    stage[koff * n + c] = ((m & 1) ? buf1 : buf0)[list[c]];
}

// Eq. psiphasor for the `count` staged steps ctr[0] .. ctr[0] + count - 1 of
// a launch group at each of nk wavenumbers, added in step order: one
// read-modify-write of the FP64 sums per group instead of per pair.  The
// group's staged values are read once, for every wavenumber; plain FP64
// sums, as in shell_dft_kernel (the compensation array stays zero).
__global__ void shell_flush_kernel(const int64_t* __restrict__ ctr, int count, const int* __restrict__ dft_tab,
                                   const double2* __restrict__ w_tab, int64_t wstride, int nk,
                                   const float2* __restrict__ stage, int64_t n, double2* __restrict__ sum) {
    const int64_t first = ctr[0];
    bool any = false;
    for (int k = 0; k < count; ++k) any |= first + k < ctr[1] && dft_tab[first + k] != 0;
    if (!any) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    // slots k < count lie inside the ring; a slot whose step is past the run's
    // end was not written this group and is skipped below
    float2 v[kStageSteps];
#pragma unroll
    for (int k = 0; k < kStageSteps; ++k) v[k] = k < count ? stage[k * n + c] : make_float2(0.f, 0.f);
    for (int f = 0; f < nk; ++f) {
        double2 s = sum[f * n + c];
#pragma unroll
        for (int k = 0; k < kStageSteps; ++k) {
            const int64_t m = first + k;
            if (k >= count || m >= ctr[1] || !dft_tab[m]) continue;
            const double2 w = w_tab[f * wstride + m];
            s.x += w.x * v[k].x - w.y * v[k].y;
            s.y += w.x * v[k].y + w.y * v[k].x;
        }
        sum[f * n + c] = s;
    }
}

// node values: separable interpolation of (sum + comp) * scale - inc (scale
// complex: one over the incident phasor)
__global__ void node_kernel(int n_nodes, const int* __restrict__ start, const double* __restrict__ lw,
                            const double3* __restrict__ normal, const int* __restrict__ slot, int nx, int ny,
                            const double2* __restrict__ sum, const double2* __restrict__ comp,
                            const double2* __restrict__ inc, double2 scale, double2* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_nodes) return;
    const int ix = start[3 * q], iy = start[3 * q + 1], iz = start[3 * q + 2];
    const double* W = lw + (int64_t)q * 3 * 2 * kStencil;
    const double* Lx = W;
    const double* dLx = W + kStencil;
    const double* Ly = W + 2 * kStencil;
    const double* dLy = W + 3 * kStencil;
    const double* Lz = W + 4 * kStencil;
    const double* dLz = W + 5 * kStencil;
    double vr = 0, vi = 0, gxr = 0, gxi = 0, gyr = 0, gyi = 0, gzr = 0, gzi = 0;
    for (int c = 0; c < kStencil; ++c) {
        for (int b = 0; b < kStencil; ++b) {
            const double wyz = Ly[b] * Lz[c], wdy = dLy[b] * Lz[c], wdz = Ly[b] * dLz[c];
            for (int a = 0; a < kStencil; ++a) {
                const int64_t lin = (ix + a) + (int64_t)nx * ((iy + b) + (int64_t)ny * (iz + c));
                const int sl = slot[lin];
                const double2 sv = sum[sl], cv = comp[sl], iv = inc[sl];
                const double ar = sv.x + cv.x, ai = sv.y + cv.y;
                const double pr = ar * scale.x - ai * scale.y - iv.x, pi = ar * scale.y + ai * scale.x - iv.y;
                const double w0 = Lx[a] * wyz;
                vr += w0 * pr;
                vi += w0 * pi;
                const double wx = dLx[a] * wyz;
                gxr += wx * pr;
                gxi += wx * pi;
                const double wy = Lx[a] * wdy;
                gyr += wy * pr;
                gyi += wy * pi;
                const double wz = Lx[a] * wdz;
                gzr += wz * pr;
                gzi += wz * pi;
            }
        }
    }
    const double3 nq = normal[q];
    out[q] = make_double2(vr, vi);
    out[n_nodes + q] = make_double2(nq.x * gxr + nq.y * gyr + nq.z * gzr, nq.x * gxi + nq.y * gyi + nq.z * gzi);
}

constexpr int kNodeChunk = 256;

// Psi(r) = -(1/4pi) sum_q w_q exp(ikR)/R [dn psi + (-ik + 1/R)(n . (s - r)/R) psi],
// k the reduced wavenumber of the phasors (1 for the central wave)
__global__ __launch_bounds__(256) void sphere_points_kernel(int n_nodes, const double3* __restrict__ node,
                                                            const double3* __restrict__ normal,
                                                            const double* __restrict__ weight,
                                                            const double2* __restrict__ ph, const double3* __restrict__ obs,
                                                            int64_t n_obs, double k0, double kw,
                                                            double2* __restrict__ out) {
    __shared__ double3 s_node[kNodeChunk], s_nrm[kNodeChunk];
    __shared__ double s_w[kNodeChunk];
    __shared__ double2 s_v[kNodeChunk], s_d[kNodeChunk];
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = o < n_obs;
    double3 r = make_double3(0, 0, 0);
    if (live) {
        const double3 p = obs[o];
        r = make_double3(p.x * k0, p.y * k0, p.z * k0);
    }
    double ar = 0, ai = 0;
    for (int q0 = 0; q0 < n_nodes; q0 += kNodeChunk) {
        const int nq = min(kNodeChunk, n_nodes - q0);
        __syncthreads();
        for (int e = threadIdx.x; e < nq; e += blockDim.x) {
            s_node[e] = node[q0 + e];
            s_nrm[e] = normal[q0 + e];
            s_w[e] = weight[q0 + e];
            s_v[e] = ph[q0 + e];
            s_d[e] = ph[n_nodes + q0 + e];
        }
        __syncthreads();
        if (!live) continue;
        for (int e = 0; e < nq; ++e) {
            const double dx = s_node[e].x - r.x, dy = s_node[e].y - r.y, dz = s_node[e].z - r.z;
            const double R = sqrt(dx * dx + dy * dy + dz * dz);
            const double inv = 1.0 / R;
            const double ndr = (s_nrm[e].x * dx + s_nrm[e].y * dy + s_nrm[e].z * dz) * inv;
            // dn psi + (-ik + 1/R) ndr psi
            const double2 v = s_v[e], d = s_d[e];
            const double tr = d.x + ndr * (kw * v.y + inv * v.x);
            const double ti = d.y + ndr * (-kw * v.x + inv * v.y);
            double sn, cs;
            sincos(kw * R, &sn, &cs);
            const double f = s_w[e] * inv;
            ar += f * (cs * tr - sn * ti);
            ai += f * (cs * ti + sn * tr);
        }
    }
    if (live) out[o] = make_double2(-ar / (4 * kPi), -ai / (4 * kPi));
}

// f(r_hat) = -(1/4pi) sum_q w_q [dn psi + ik (n . r_hat) psi] exp(-ik r_hat . s) / k0
__global__ __launch_bounds__(256) void sphere_far_kernel(int n_nodes, const double3* __restrict__ node,
                                                         const double3* __restrict__ normal,
                                                         const double* __restrict__ weight,
                                                         const double2* __restrict__ ph, const double3* __restrict__ dirs,
                                                         int64_t n_dir, double k0, double kw,
                                                         double2* __restrict__ out) {
    __shared__ double3 s_node[kNodeChunk], s_nrm[kNodeChunk];
    __shared__ double s_w[kNodeChunk];
    __shared__ double2 s_v[kNodeChunk], s_d[kNodeChunk];
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = o < n_dir;
    double3 rh = make_double3(0, 0, 1);
    if (live) rh = dirs[o];
    double ar = 0, ai = 0;
    for (int q0 = 0; q0 < n_nodes; q0 += kNodeChunk) {
        const int nq = min(kNodeChunk, n_nodes - q0);
        __syncthreads();
        for (int e = threadIdx.x; e < nq; e += blockDim.x) {
            s_node[e] = node[q0 + e];
            s_nrm[e] = normal[q0 + e];
            s_w[e] = weight[q0 + e];
            s_v[e] = ph[q0 + e];
            s_d[e] = ph[n_nodes + q0 + e];
        }
        __syncthreads();
        if (!live) continue;
        for (int e = 0; e < nq; ++e) {
            const double nr = s_nrm[e].x * rh.x + s_nrm[e].y * rh.y + s_nrm[e].z * rh.z;
            const double2 v = s_v[e], d = s_d[e];
            const double tr = d.x - kw * nr * v.y, ti = d.y + kw * nr * v.x;  // dn psi + ik nr psi
            double sn, cs;
            sincos(-kw * (rh.x * s_node[e].x + rh.y * s_node[e].y + rh.z * s_node[e].z), &sn, &cs);
            ar += s_w[e] * (cs * tr - sn * ti);
            ai += s_w[e] * (cs * ti + sn * tr);
        }
    }
    if (live) out[o] = make_double2(-ar / (4 * kPi * k0), -ai / (4 * kPi * k0));
}

}  // namespace

void sphere_free(SphereState* sp) {
    if (!sp) return;
    void* ptrs[] = {sp->node, sp->normal, sp->weight, sp->start, sp->lw,   sp->list,
                    sp->slot, sp->inc,    sp->sum,    sp->comp,  sp->phasor, sp->stage};
    for (void* p : ptrs) (void)hipFree(p);
    delete sp;
}

pstd_status sphere_create(pstd_solver* s) {
    const pstd_problem& p = s->prob;
    if (p.surface_kind == 0) return PSTD_OK;
    if (p.surface_kind != 1) return solver_fail(s, PSTD_EINVAL, "surface_kind must be 0 (box) or 1 (sphere)");
    if (!(p.sphere_radius > 0)) return solver_fail(s, PSTD_EINVAL, "sphere_radius must be positive");
    const int nth = p.sphere_nodes[0] > 0 ? p.sphere_nodes[0] : 64;
    const int nph = p.sphere_nodes[1] > 0 ? p.sphere_nodes[1] : 128;
    if (p.sphere_nodes[0] < 0 || p.sphere_nodes[1] < 0 || nth < 2 || nph < 3)
        return solver_fail(s, PSTD_EINVAL, "sphere_nodes must be positive (theta >= 2, phi >= 3)");
    // the sphere must enclose the region where the taper is one
    for (int c = 0; c < 8; ++c) {
        double r2 = 0;
        for (int a = 0; a < 3; ++a) {
            const int idx = (c >> a & 1) ? p.tfsf[a][2] : p.tfsf[a][1];
            const double x = (idx - p.n[a] / 2) * p.h[a];
            r2 += x * x;
        }
        if (std::sqrt(r2) >= p.sphere_radius)
            return solver_fail(s, PSTD_EINVAL, "the sphere must enclose the region where the taper is one");
    }
    const int nx = p.n[0], ny = p.n[1];
    const int n_nodes = nth * nph;
    std::vector<double> ct, wt;
    gauss_legendre(nth, ct, wt);
    std::vector<double3> node(n_nodes), nrm(n_nodes);
    std::vector<double> weight(n_nodes);
    std::vector<int> start(3 * (size_t)n_nodes);
    std::vector<double> lw((size_t)n_nodes * 3 * 2 * kStencil);
    std::vector<char> used(s->cells, 0);
    const double R = p.sphere_radius * p.k0;
    for (int i = 0; i < nth; ++i)
        for (int j = 0; j < nph; ++j) {
            const int q = i * nph + j;
            const double st = std::sqrt(1 - ct[i] * ct[i]), ph = 2 * kPi * j / nph;
            nrm[q] = make_double3(st * std::cos(ph), st * std::sin(ph), ct[i]);
            node[q] = make_double3(R * nrm[q].x, R * nrm[q].y, R * nrm[q].z);
            weight[q] = R * R * wt[i] * 2 * kPi / nph;
            const double c3[3] = {node[q].x, node[q].y, node[q].z};
            for (int a = 0; a < 3; ++a) {
                const double u = c3[a] / s->dxb[a] + p.n[a] / 2;
                double* W = &lw[((size_t)q * 3 + a) * 2 * kStencil];
                const int i0 = lagrange(u, W, W + kStencil);
                for (int m = 0; m < kStencil; ++m) W[kStencil + m] /= s->dxb[a];  // per reduced length
                // stencil inside the grid and outside the absorber
                if (i0 < p.abc_cells[a] || i0 + kStencil > p.n[a] - p.abc_cells[a])
                    return solver_fail(s, PSTD_EINVAL, "the sphere's interpolation shell reaches the absorber");
                start[3 * (size_t)q + a] = i0;
            }
            const int* st3 = &start[3 * (size_t)q];
            for (int c = 0; c < kStencil; ++c)
                for (int b = 0; b < kStencil; ++b)
                    for (int a = 0; a < kStencil; ++a)
                        used[(st3[0] + a) + (int64_t)nx * ((st3[1] + b) + (int64_t)ny * (st3[2] + c))] = 1;
        }
    std::vector<int> list, slot(s->cells, -1);
    for (int64_t c = 0; c < s->cells; ++c)
        if (used[c]) {
            slot[c] = (int)list.size();
            list.push_back((int)c);
        }
    std::vector<double2> ia[3];
    for (int a = 0; a < 3; ++a) solver_incident_axis(s, a, ia[a]);
    std::vector<double2> inc(list.size());
    for (size_t k = 0; k < list.size(); ++k) {
        const int64_t c = list[k];
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), kz = (int)(c / ((int64_t)nx * ny));
        const double2 x = ia[0][i], y = ia[1][j], z = ia[2][kz];
        const double2 xy = make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
        inc[k] = make_double2(xy.x * z.x - xy.y * z.y, xy.x * z.y + xy.y * z.x);
    }
    // |exp(i khat . x)| = 1, so |inc| is the taper on the shell
    double inc_max = 0;
    for (const double2& v : inc) inc_max = std::max(inc_max, std::sqrt(v.x * v.x + v.y * v.y));
    SphereState* sp = new SphereState();
    s->sphere = sp;
    sp->n_nodes = n_nodes;
    sp->R = R;
    sp->n_shell = (int64_t)list.size();
    sp->inc_max = inc_max;
    hipError_t e;
    auto up = [&](auto** dst, const auto& v) {
        using T = typename std::decay_t<decltype(v)>::value_type;
        hipError_t r = hipMalloc((void**)dst, v.size() * sizeof(T));
        if (r == hipSuccess) r = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        return r;
    };
    if ((e = up(&sp->node, node)) || (e = up(&sp->normal, nrm)) || (e = up(&sp->weight, weight)) ||
        (e = up(&sp->start, start)) || (e = up(&sp->lw, lw)) || (e = up(&sp->list, list)) ||
        (e = up(&sp->slot, slot)) || (e = up(&sp->inc, inc)) ||
        (e = hipMalloc(&sp->sum, sp->n_shell * sizeof(double2))) ||
        (e = hipMalloc(&sp->comp, sp->n_shell * sizeof(double2))) ||
        (e = hipMalloc(&sp->phasor, 2 * (size_t)n_nodes * sizeof(double2))) ||
        (e = hipMemset(sp->sum, 0, sp->n_shell * sizeof(double2))) ||
        (e = hipMemset(sp->comp, 0, sp->n_shell * sizeof(double2))))
        return solver_hip_fail(s, e, "sphere tables");
    return PSTD_OK;
}

hipError_t sphere_launch_dft(const pstd_solver* s, int koff, int count, hipStream_t stream) {
    const SphereState* sp = s->sphere;
    if (!sp || sp->n_shell == 0 || count < 1) return hipSuccess;
    if (count > 2 || koff < count - 1) return hipErrorInvalidValue;
    if (sp->nk != 1) return hipErrorInvalidValue;  // several wavenumbers are staged
    hipLaunchKernelGGL(shell_dft_kernel, dim3((unsigned)((sp->n_shell + 255) / 256)), dim3(256), 0, stream, s->ctr,
                       koff, count, s->dft_tab, s->w_tab, s->buf[0], s->buf[1], sp->list, sp->n_shell, sp->sum);
    return hipGetLastError();
}

bool sphere_staged(const pstd_solver* s) { return s->sphere && s->sphere->stage; }

void sphere_drop_stage(pstd_solver* s) {
    if (!s->sphere) return;
    (void)hipFree(s->sphere->stage);
    s->sphere->stage = nullptr;
}

void sphere_stage_buffers(const pstd_solver* s, const int** list, int64_t* n_shell, float2** stage) {
    const SphereState* sp = s->sphere;
    *list = sp ? sp->list : nullptr;
    *n_shell = sp ? sp->n_shell : 0;
    *stage = sp ? sp->stage : nullptr;
}

hipError_t sphere_launch_stage(const pstd_solver* s, int koff, hipStream_t stream) {
    const SphereState* sp = s->sphere;
    if (!sp || !sp->stage || sp->n_shell == 0) return hipSuccess;
    if (koff < 0 || koff >= kStageSteps) return hipErrorInvalidValue;
    hipLaunchKernelGGL(shell_stage_kernel, dim3((unsigned)((sp->n_shell + 255) / 256)), dim3(256), 0, stream, s->ctr,
                       koff, s->buf[0], s->buf[1], sp->list, sp->n_shell, sp->stage);
    return hipGetLastError();
}

hipError_t sphere_launch_flush(const pstd_solver* s, int count, hipStream_t stream) {
    const SphereState* sp = s->sphere;
    if (!sp || !sp->stage || sp->n_shell == 0) return hipSuccess;
    if (count < 1 || count > kStageSteps) return hipErrorInvalidValue;
    hipLaunchKernelGGL(shell_flush_kernel, dim3((unsigned)((sp->n_shell + 255) / 256)), dim3(256), 0, stream, s->ctr,
                       count, s->dft_tab, s->w_tab, s->tab_cap, sp->nk, sp->stage, sp->n_shell, sp->sum);
    return hipGetLastError();
}

hipError_t sphere_clear(pstd_solver* s, hipStream_t stream) {
    SphereState* sp = s->sphere;
    if (!sp) return hipSuccess;
    const size_t b = sp->nk * sp->n_shell * sizeof(double2);
    hipError_t e = hipMemsetAsync(sp->sum, 0, b, stream);
    if (e == hipSuccess) e = hipMemsetAsync(sp->comp, 0, b, stream);
    return e;
}

hipError_t sphere_set_wavenumbers(pstd_solver* s, int nk) {
    SphereState* sp = s->sphere;
    if (!sp || nk < 1) return hipErrorInvalidValue;
    (void)hipFree(sp->sum);
    (void)hipFree(sp->comp);
    (void)hipFree(sp->stage);
    sp->sum = sp->comp = nullptr;
    sp->stage = nullptr;
    sp->nk = nk;
    const size_t b = nk * sp->n_shell * sizeof(double2);
    hipError_t e = hipMalloc(&sp->sum, b);
    if (e == hipSuccess) e = hipMalloc(&sp->comp, b);
    if (e == hipSuccess) e = hipMalloc(&sp->stage, kStageSteps * sp->n_shell * sizeof(float2));
    if (e == hipSuccess) e = hipMemset(sp->sum, 0, b);
    if (e == hipSuccess) e = hipMemset(sp->comp, 0, b);
    return e;
}

double sphere_taper_max(const pstd_solver* s) { return s->sphere ? s->sphere->inc_max : 0.0; }

int64_t sphere_state_bytes(const pstd_solver* s) {
    return s->sphere ? 2 * s->sphere->nk * s->sphere->n_shell * (int64_t)sizeof(double2) : 0;
}

hipError_t sphere_save(const pstd_solver* s, char* dst, hipStream_t stream) {
    const SphereState* sp = s->sphere;
    if (!sp) return hipSuccess;
    const size_t b = sp->nk * sp->n_shell * sizeof(double2);
    hipError_t e = hipMemcpyAsync(dst, sp->sum, b, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dst + b, sp->comp, b, hipMemcpyDeviceToDevice, stream);
    return e;
}

hipError_t sphere_load(pstd_solver* s, const char* src, hipStream_t stream) {
    SphereState* sp = s->sphere;
    if (!sp) return hipSuccess;
    const size_t b = sp->nk * sp->n_shell * sizeof(double2);
    hipError_t e = hipMemcpyAsync(sp->sum, src, b, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sp->comp, src + b, b, hipMemcpyDeviceToDevice, stream);
    return e;
}

int64_t sphere_nodes(const pstd_solver* s) { return s->sphere ? s->sphere->n_nodes : 0; }

hipError_t sphere_phasors(pstd_solver* s, const SphereOut& o, double2* out, hipStream_t stream) {
    SphereState* sp = s->sphere;
    if (o.ik < 0 || o.ik >= sp->nk) return hipErrorInvalidValue;
    const int64_t off = (int64_t)o.ik * sp->n_shell;
    hipLaunchKernelGGL(node_kernel, dim3((unsigned)((sp->n_nodes + 127) / 128)), dim3(128), 0, stream, sp->n_nodes,
                       sp->start, sp->lw, sp->normal, sp->slot, s->prob.n[0], s->prob.n[1], sp->sum + off,
                       sp->comp + off, sp->inc, o.scale, sp->phasor);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, sp->phasor, 2 * (size_t)sp->n_nodes * sizeof(double2), hipMemcpyDeviceToDevice, stream);
    return e;
}

hipError_t sphere_project(pstd_solver* s, const SphereOut& o, const double3* obs, int64_t n_obs, double2* out,
                          hipStream_t stream) {
    SphereState* sp = s->sphere;
    hipError_t e = sphere_phasors(s, o, nullptr, stream);
    if (e || n_obs == 0) return e;
    hipLaunchKernelGGL(sphere_points_kernel, dim3((unsigned)((n_obs + 255) / 256)), dim3(256), 0, stream, sp->n_nodes,
                       sp->node, sp->normal, sp->weight, sp->phasor, obs, n_obs, s->prob.k0, o.k, out);
    return hipGetLastError();
}

hipError_t sphere_far_field(pstd_solver* s, const SphereOut& o, const double3* dirs, int64_t n_dir, double2* out,
                            hipStream_t stream) {
    SphereState* sp = s->sphere;
    hipError_t e = sphere_phasors(s, o, nullptr, stream);
    if (e || n_dir == 0) return e;
    hipLaunchKernelGGL(sphere_far_kernel, dim3((unsigned)((n_dir + 255) / 256)), dim3(256), 0, stream, sp->n_nodes,
                       sp->node, sp->normal, sp->weight, sp->phasor, dirs, n_dir, s->prob.k0, o.k, out);
    return hipGetLastError();
}

}  // namespace pstd
