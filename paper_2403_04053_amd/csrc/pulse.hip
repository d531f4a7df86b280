// Pulsed incidence (Section 2.2.3, calculation of the incident wave; Section
// 3.3 at several frequencies).  A plane-wave packet of any shape travels
// along k_hat; cells on one wavefront share its value, so the packet is a 1D
// problem on the axis that starts at the corner of the taper box the front
// meets first (Eq. Oinc), a cell sitting at d = k_hat . (x - x_O) on it (Eq.
// inc_d).  The packet is stepped in free space by the 3D model's leapfrog in
// 1D; in the spectral basis every mode is independent, so step n of the
// leapfrog started on each mode's physical root is exactly
//   a_l(n) = c_l exp(-i theta_l n),  sin(theta_l) = dtau eta k_l^2,
// c_l = F[psi^0]_l / N, and nothing has to be stored per step.
//
// Before the passes of each step, one launch (pulse_pre_kernel) evaluates
// the spectral interpolation of Eqs. pstd_psiinc / pstd_dpsiinc for the next
// step on a table four times finer than the grids, over the d-range of the
// transition layer only (a few hundred points, one wave each), interpolates
// this step's table at every layer cell with 8-point Lagrange weights (error
// ~ (k h)^8 / 8!, below 1e-8 of the packet) and adds the layer source of Eq.
// dimlesstildeSchrodinger, lap(zeta) psi_inc + 2 grad(zeta) . k_hat
// dpsi_inc/dd, times -i 2 dtau (eta), to psi^{n-1} before the z pass, which
// multiplies it by Gamma: the update is linear, so this equals adding it
// inside.  The passes are unchanged; the monochromatic source is off
// (sigma = 0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "solver.hpp"

namespace pstd {

struct PulseState {
    int K = 0;                 // modes l_lo .. l_lo + K - 1
    double k_lo = 0, dk = 0;   // k_l = k_lo + (l - l_lo) dk
    double2* coef = nullptr;   // c_l
    double* theta = nullptr;   // phase per step of each mode
    int J = 0;                 // table points d_lo + j h
    double d_lo = 0, h = 0;
    double2* tab = nullptr;    // [step parity][2][J]: sum a_l e^{i k_l d}, sum a_l k_l e^{i k_l d}
    double2* ekd = nullptr;    // [J][K]: e^{i k_l d_j}
    int64_t n_cells = 0;       // transition-layer cells
    int* cell = nullptr;
    int* j0 = nullptr;         // first table point of each cell's stencil
    double* w = nullptr;       // [cell][8] Lagrange weights
    double2* ab = nullptr;     // per cell: Gamma fac lap(zeta), Gamma fac 2 grad(zeta) . k_hat
    // host
    std::vector<double> kbar, W;        // wavenumbers of the phasors and their frequencies
    std::vector<double2> g;             // c_l exp(i k_l d_origin)
    std::vector<double> theta_h;
    int64_t from = 0;                   // first step since creation or pstd_set_state
    // box surface: the passes stage the plane values of a launch group, the
    // flush adds them to one set of plane sums per wavenumber
    bool box = false;
    float2* bstage[3] = {nullptr, nullptr, nullptr};  // [group step][side][psi, dpsi][points]
    double2* bacc[3] = {nullptr, nullptr, nullptr};   // [wavenumber][side][4][points], as PassArgs::acc
    std::vector<ProjectState*> proj;                  // box projection per wavenumber
};

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kLag = 8;
constexpr int kModeChunk = 256;

// compensated (Neumaier) summation step
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

// in-place radix-2 DFT, forward (e^{-i 2 pi l j / N}), N a power of two
void fft_pow2(std::vector<std::complex<double>>& a) {
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const double ang = -2 * kPi * (double)k / (double)len;
                const std::complex<double> w(std::cos(ang), std::sin(ang));
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

// One launch before the passes of step n = ctr[0] + koff, three kinds of
// blocks, each touching its own buffers:
//  * table blocks: T0(d_j) = sum_l a_l(m) e^{i k_l d_j} and T1(d_j) = sum_l
//    a_l(m) k_l e^{i k_l d_j} for the next step m = n + 1, into the table
//    buffer of m's parity.  One wave per table point: its 64 lanes take
//    every 64th mode (a_l(m) shared by the block's four points through LDS,
//    e^{i k_l d_j} from the precomputed table), then the wave adds the lane
//    sums in a fixed order;
//  * source blocks: the layer source of step n from the table of n's parity
//    (interpolated with the cell's 8 Lagrange weights), -i fac S added to
//    psi^{n-1}, which only the z pass reads next and which it multiplies by
//    Gamma: the same as adding -i Gamma fac S inside the update;
//  * stage blocks: psi^n on the sphere's shell into slot koff of the ring.
// koff = -1 with table blocks only primes the table of step ctr[0].
__global__ __launch_bounds__(256) void pulse_pre_kernel(const int64_t* __restrict__ ctr, int koff, int K,
                                                        const double2* __restrict__ coef,
                                                        const double* __restrict__ theta, double k_lo, double dk,
                                                        int J, const double2* __restrict__ ekd,
                                                        double2* __restrict__ tab, int table_blocks,
                                                        int64_t nc, const int* __restrict__ cell,
                                                        const int* __restrict__ j0, const double* __restrict__ w,
                                                        const double2* __restrict__ ab, int source_blocks,
                                                        float2* __restrict__ buf0, float2* __restrict__ buf1,
                                                        const int* __restrict__ list, int64_t n_shell,
                                                        float2* __restrict__ stage) {
    // the launch is bound by latency: what does not depend on the step (the
    // cell and shell indices, the stencil weights) is loaded before the
    // step counter, so that those loads and the counter's are in flight
    // together
    const int blk = (int)blockIdx.x;
    if (blk >= table_blocks + source_blocks) {
        const int64_t c = (int64_t)(blk - table_blocks - source_blocks) * blockDim.x + threadIdx.x;
        if (c >= n_shell) return;
        const int src = list[c];
        const int64_t n = ctr[0] + koff;
        if (n >= ctr[1]) return;
        stage[koff * n_shell + c] = ((n & 1) ? buf1 : buf0)[src];
        return;
    }
    if (blk >= table_blocks) {
        const int64_t c = (int64_t)(blk - table_blocks) * blockDim.x + threadIdx.x;
        if (c >= nc) return;
        const int j = j0[c];
        const int cc = cell[c];
        const double2 q = ab[c];
        double wc[kLag];
        for (int m = 0; m < kLag; ++m) wc[m] = w[kLag * c + m];
        const int64_t n = ctr[0] + koff;
        if (n >= ctr[1]) return;
        const double2* t = tab + (n & 1) * 2 * (int64_t)J;
        double p0r = 0, p0i = 0, p1r = 0, p1i = 0;
        for (int m = 0; m < kLag; ++m) {
            const double2 t0 = t[j + m], t1 = t[J + j + m];
            p0r += wc[m] * t0.x;
            p0i += wc[m] * t0.y;
            p1r += wc[m] * t1.x;
            p1i += wc[m] * t1.y;
        }
        // S = A T0 + B i T1; psi^{n-1} -= i S
        const double sr = q.x * p0r - q.y * p1i, si = q.x * p0i + q.y * p1r;
        float2* out = ((n + 1) & 1) ? buf1 : buf0;
        float2 v = out[cc];
        v.x += (float)si;
        v.y -= (float)sr;
        out[cc] = v;
        return;
    }
    // the next step's mode amplitudes a_l(m) = c_l e^{-i theta_l m}, once per
    // block in LDS (chunks of kModeChunk = blockDim.x modes, one per thread);
    // every wave of a table block takes part in the barriers, those past the
    // table's end store nothing.  Each chunk's operands (the wave's row of
    // e^{i k_l d_j}, theta_l, c_l) are loaded before anything waits: the
    // first chunk's before the step counter is read.
    constexpr int kPer = kModeChunk / 64;
    __shared__ double2 a_s[kModeChunk];
    const int lane = threadIdx.x & 63;
    const int jt = blk * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const double2* e_j = ekd + (int64_t)min(jt, J - 1) * K;
    double2 ev[kPer];
    double th = 0;
    double2 cf = make_double2(0, 0);
    auto load_chunk = [&](int m0, int nm) {
        for (int i = 0; i < kPer; ++i) {
            const int l = lane + 64 * i;
            ev[i] = l < nm ? e_j[m0 + l] : make_double2(0, 0);
        }
        if ((int)threadIdx.x < nm) {
            th = theta[m0 + threadIdx.x];
            cf = coef[m0 + threadIdx.x];
        }
    };
    load_chunk(0, min(kModeChunk, K));
    const int64_t n = ctr[0] + koff;
    if (n >= ctr[1]) return;
    const int64_t mstep = n + 1;
    double s0r = 0, s0i = 0, s1r = 0, s1i = 0;
    for (int m0 = 0; m0 < K; m0 += kModeChunk) {
        const int nm = min(kModeChunk, K - m0);
        if (m0 > 0) load_chunk(m0, nm);
        __syncthreads();
        if ((int)threadIdx.x < nm) {
            double sn, cs;
            sincos(th * (double)mstep, &sn, &cs);
            a_s[threadIdx.x] = make_double2(cf.x * cs + cf.y * sn, cf.y * cs - cf.x * sn);
        }
        __syncthreads();
        for (int i = 0; i < kPer; ++i) {
            const int l = lane + 64 * i;
            if (l < nm) {
                const double2 a = a_s[l], e = ev[i];
                const double tr = a.x * e.x - a.y * e.y, ti = a.x * e.y + a.y * e.x;
                const double kl = k_lo + (m0 + l) * dk;
                s0r += tr;
                s0i += ti;
                s1r += kl * tr;
                s1i += kl * ti;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        s0r += __shfl_xor(s0r, off);
        s0i += __shfl_xor(s0i, off);
        s1r += __shfl_xor(s1r, off);
        s1i += __shfl_xor(s1i, off);
    }
    if (lane == 0 && jt < J) {
        double2* t = tab + (mstep & 1) * 2 * (int64_t)J;
        t[jt] = make_double2(s0r, s0i);
        t[J + jt] = make_double2(s1r, s1i);
    }
}

// the staged plane values of the launch group's steps ctr[0] .. ctr[0] +
// count - 1 into the FP64 plane sums of each wavenumber, in step order; one
// thread per (side, field, plane point)
// the three axes' staged plane values and sums, one launch for all
struct BoxFlush {
    const float2* stage[3];
    double2* acc[3];
    int64_t points[3];
    int blocks[3];
};

// one thread per (wavenumber, side, field, plane point): the group's staged
// values are loaded before the step counter is read, then added in step
// order to the compensated sums
__global__ __launch_bounds__(256) void box_flush_kernel(const int64_t* __restrict__ ctr, int count,
                                                        const int* __restrict__ dft_tab,
                                                        const double2* __restrict__ w_tab, int64_t wstride, int nk,
                                                        BoxFlush bf) {
    int b = (int)blockIdx.x, a = 0;
    while (a < 2 && b >= bf.blocks[a]) b -= bf.blocks[a++];
    const int64_t points = bf.points[a];
    const int64_t i = (int64_t)b * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nk * 4 * points) return;
    const int f = (int)(i / (4 * points));
    const int64_t r = i - (int64_t)f * 4 * points;
    const int sf = (int)(r / points);  // side * 2 + field
    const int64_t pt = r - (int64_t)sf * points;
    float2 v[kStageSteps];
#pragma unroll
    for (int k = 0; k < kStageSteps; ++k)
        v[k] = k < count ? bf.stage[a][((int64_t)k * 4 + sf) * points + pt] : make_float2(0.f, 0.f);
    double2* S = bf.acc[a] + ((int64_t)f * 8 + (sf >> 1) * 4 + (sf & 1) * 2) * points + pt;
    double2* Cc = S + points;
    double2 s = *S, c = *Cc;
    const int64_t first = ctr[0], end = ctr[1];
    bool any = false;
#pragma unroll
    for (int k = 0; k < kStageSteps; ++k) {
        const int64_t m = first + k;
        if (k >= count || m >= end || !dft_tab[m]) continue;
        any = true;
        const double2 w = w_tab[f * wstride + m];
        neumaier(s.x, c.x, w.x * v[k].x - w.y * v[k].y);
        neumaier(s.y, c.y, w.x * v[k].y + w.y * v[k].x);
    }
    if (any) {
        *S = s;
        *Cc = c;
    }
}

}  // namespace

void pulse_free(PulseState* p) {
    if (!p) return;
    void* ptrs[] = {p->coef, p->theta, p->tab, p->ekd, p->cell, p->j0, p->w, p->ab,
                    p->bstage[0], p->bstage[1], p->bstage[2], p->bacc[0], p->bacc[1], p->bacc[2]};
    for (void* q : ptrs) (void)hipFree(q);
    for (ProjectState* q : p->proj) project_free(q);
    delete p;
}

int pulse_wavenumbers(const pstd_solver* s) { return s->pulse ? (int)s->pulse->kbar.size() : 1; }

int64_t pulse_from(const pstd_solver* s) { return s->pulse ? s->pulse->from : 0; }

double pulse_frequency(const pstd_solver* s, int ik) { return s->pulse ? s->pulse->W[ik] : s->omega; }

pstd_status pulse_set(pstd_solver* s, const double* psi0, int32_t n1d, double delta, const double* kbar, int32_t nk) {
    const pstd_problem& p = s->prob;
    if (s->in_batch) return solver_fail(s, PSTD_EUNSUPPORTED, "batch instances take the monochromatic wave only");
    if (p.scheme != 0 || p.sub_core[0] || p.sub_core[1] || p.sub_core[2])
        return solver_fail(s, PSTD_EUNSUPPORTED, "pulsed incidence needs the spectral scheme and no subdomains");
    const bool box = p.surface_kind == 0;
    if (s->step != 0 || s->win_steps != 0) return solver_fail(s, PSTD_ESTATE, "set the pulse before the first step");
    if (!psi0 || !kbar) return solver_fail(s, PSTD_EINVAL, "null pulse or wavenumber array");
    if (n1d < 8 || n1d > (1 << 20) || (n1d & (n1d - 1)))
        return solver_fail(s, PSTD_EINVAL, "n1d must be a power of two in [8, 2^20]");
    if (!(delta > 0) || !std::isfinite(delta)) return solver_fail(s, PSTD_EINVAL, "delta must be positive");
    if (nk < 1 || nk > 64) return solver_fail(s, PSTD_EINVAL, "1 to 64 wavenumbers");
    if (!box && sphere_taper_max(s) != 0)
        return solver_fail(s, PSTD_EINVAL, "the sphere's shell must lie where the taper is zero");
    for (int a = 0; a < 3 && box; ++a)
        if (!(p.surf_lo[a] <= p.tfsf[a][0] && p.surf_hi[a] >= p.tfsf[a][3]))
            return solver_fail(s, PSTD_EINVAL, "the box planes must lie where the taper is zero");
    const double q = s->dtau * s->eta;
    const double knyq = kPi / delta;
    if (!(q * knyq * knyq < 1)) return solver_fail(s, PSTD_EINVAL, "the 1D grid's Nyquist mode exceeds the step bound");
    std::vector<double> W(nk);
    for (int f = 0; f < nk; ++f) {
        if (!(kbar[f] > 0) || !(q * kbar[f] * kbar[f] < 1))
            return solver_fail(s, PSTD_EINVAL, "wavenumbers must be positive and below the step bound");
        W[f] = std::asin(q * kbar[f] * kbar[f]) / s->dtau;
    }
    // spectrum of the packet
    std::vector<std::complex<double>> F(n1d);
    double amax = 0;
    for (int j = 0; j < n1d; ++j) {
        if (!std::isfinite(psi0[2 * j]) || !std::isfinite(psi0[2 * j + 1]))
            return solver_fail(s, PSTD_EINVAL, "the pulse is not finite");
        F[j] = {psi0[2 * j], psi0[2 * j + 1]};
    }
    fft_pow2(F);
    for (auto& v : F) {
        v /= (double)n1d;
        amax = std::max(amax, std::abs(v));
    }
    if (!(amax > 0)) return solver_fail(s, PSTD_EINVAL, "the pulse is zero");
    // contiguous range of signed mode indices holding every mode above 1e-14 of the largest
    int lmin = n1d, lmax = -n1d;
    for (int j = 0; j < n1d; ++j) {
        const int l = j >= n1d / 2 ? j - n1d : j;
        if (std::abs(F[j]) > 1e-14 * amax) {
            lmin = std::min(lmin, l);
            lmax = std::max(lmax, l);
        }
    }
    const int K = lmax - lmin + 1;
    const double dk = 2 * kPi / (n1d * delta);
    PulseState* ps = new PulseState();
    ps->K = K;
    ps->dk = dk;
    ps->k_lo = lmin * dk;
    ps->kbar.assign(kbar, kbar + nk);
    ps->W = W;
    std::vector<double2> coef(K);
    ps->theta_h.resize(K);
    for (int m = 0; m < K; ++m) {
        const int l = lmin + m;
        const std::complex<double> c = F[(l + n1d) % n1d];
        coef[m] = make_double2(c.real(), c.imag());
        const double kl = l * dk;
        ps->theta_h[m] = std::asin(q * kl * kl);
    }
    // origin corner (Eq. Oinc) and the grid origin on the axis
    int O[3];
    for (int a = 0; a < 3; ++a) O[a] = s->kh[a] >= 0 ? p.tfsf[a][0] : p.tfsf[a][3];
    double d_origin = 0;
    for (int a = 0; a < 3; ++a) d_origin += (p.n[a] / 2 - O[a]) * s->dxb[a] * s->kh[a];
    ps->g.resize(K);
    for (int m = 0; m < K; ++m) {
        const double kl = ps->k_lo + m * dk, ph = kl * d_origin;
        const double cr = std::cos(ph), ci = std::sin(ph);
        ps->g[m] = make_double2(coef[m].x * cr - coef[m].y * ci, coef[m].x * ci + coef[m].y * cr);
    }
    // transition-layer cells (taper box of every axis), their axis coordinate and coefficients
    std::vector<double> z[3], z1[3], z2[3];
    for (int a = 0; a < 3; ++a) {
        const int N = p.n[a];
        z[a].resize(N);
        z1[a].resize(N);
        z2[a].resize(N);
        for (int i = 0; i < N; ++i) solver_taper(p, a, s->dxb[a], i, &z[a][i], &z1[a][i], &z2[a][i]);
    }
    const double fac = 2.0 * s->dtau * (p.eta_on_source ? s->eta : 1.0);
    std::vector<int> cell;
    std::vector<double> dc;
    std::vector<double2> ab;
    const int64_t nx = p.n[0], ny = p.n[1];
    for (int k = p.tfsf[2][0]; k <= p.tfsf[2][3]; ++k)
        for (int j = p.tfsf[1][0]; j <= p.tfsf[1][3]; ++j)
            for (int i = p.tfsf[0][0]; i <= p.tfsf[0][3]; ++i) {
                const int ix[3] = {i, j, k};
                double lap = 0, grad = 0;
                for (int a = 0; a < 3; ++a) {
                    double others = 1;
                    for (int b = 0; b < 3; ++b)
                        if (b != a) others *= z[b][ix[b]];
                    lap += z2[a][ix[a]] * others;
                    grad += z1[a][ix[a]] * s->kh[a] * others;
                }
                if (lap == 0 && grad == 0) continue;
                cell.push_back((int)(i + nx * (j + ny * (int64_t)k)));
                double d = 0;
                for (int a = 0; a < 3; ++a) d += (ix[a] - O[a]) * s->dxb[a] * s->kh[a];
                dc.push_back(d);
                ab.push_back(make_double2(fac * lap, fac * 2.0 * grad));
            }
    ps->n_cells = (int64_t)cell.size();
    // table over the layer's d-range, 4 times finer than the finer of the two grids
    double dmin = 0, dmax = 0;
    if (!dc.empty()) {
        dmin = *std::min_element(dc.begin(), dc.end());
        dmax = *std::max_element(dc.begin(), dc.end());
    }
    ps->h = std::min(delta, std::min(s->dxb[0], std::min(s->dxb[1], s->dxb[2]))) / 4;
    ps->d_lo = dmin - 4 * ps->h;
    ps->J = (int)std::ceil((dmax - ps->d_lo) / ps->h) + 5;
    if ((int64_t)ps->J * K > (int64_t(1) << 26)) {
        pulse_free(ps);
        return solver_fail(s, PSTD_EINVAL, "the packet's spectrum is too wide for the layer's table (J K > 2^26)");
    }
    std::vector<double2> ekd((size_t)ps->J * K);
    for (int j = 0; j < ps->J; ++j)
        for (int m = 0; m < K; ++m) {
            const double ph = (ps->k_lo + m * dk) * (ps->d_lo + j * ps->h);
            ekd[(size_t)j * K + m] = make_double2(std::cos(ph), std::sin(ph));
        }
    std::vector<int> j0(cell.size());
    std::vector<double> w(kLag * cell.size());
    for (size_t c = 0; c < cell.size(); ++c) {
        const double u = (dc[c] - ps->d_lo) / ps->h;
        const int first = (int)std::floor(u) - (kLag / 2 - 1);
        j0[c] = first;
        for (int m = 0; m < kLag; ++m) {
            double l = 1;
            for (int r = 0; r < kLag; ++r)
                if (r != m) l *= (u - (first + r)) / (double)(m - r);
            w[kLag * c + m] = l;
        }
    }
    auto up = [&](auto** dst, const auto& v) {
        using T = typename std::decay_t<decltype(v)>::value_type;
        hipError_t r = hipMalloc((void**)dst, std::max<size_t>(v.size(), 1) * sizeof(T));
        if (r == hipSuccess && !v.empty()) r = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        return r;
    };
    hipError_t e;
    ps->box = box;
    ps->proj.assign(nk, nullptr);
    for (int a = 0; a < 3 && box; ++a) {
        const size_t sb = (size_t)kStageSteps * 4 * s->points[a] * sizeof(float2);
        const size_t ab_ = (size_t)nk * 8 * s->points[a] * sizeof(double2);
        if ((e = hipMalloc(&ps->bstage[a], sb)) || (e = hipMalloc(&ps->bacc[a], ab_)) ||
            (e = hipMemset(ps->bacc[a], 0, ab_))) {
            pulse_free(ps);
            return solver_hip_fail(s, e, "pulse plane sums");
        }
    }
    if ((e = hipStreamSynchronize(s->stream)) || (e = up(&ps->coef, coef)) || (e = up(&ps->theta, ps->theta_h)) ||
        (e = hipMalloc(&ps->tab, 4 * (size_t)ps->J * sizeof(double2))) || (e = up(&ps->ekd, ekd)) ||
        (e = up(&ps->cell, cell)) ||
        (e = up(&ps->j0, j0)) || (e = up(&ps->w, w)) || (e = up(&ps->ab, ab))) {
        pulse_free(ps);
        return solver_hip_fail(s, e, "pulse tables");
    }
    pulse_free(s->pulse);
    s->pulse = ps;
    if (!box && (e = sphere_set_wavenumbers(s, nk))) {
        // leave the solver as it was created: no pulse, one wavenumber
        pulse_free(s->pulse);
        s->pulse = nullptr;
        (void)sphere_set_wavenumbers(s, 1);
        sphere_drop_stage(s);
        return solver_hip_fail(s, e, "phasor sums");
    }
    // rebuild the per-step tables: no monochromatic source, one DFT weight row per wavenumber
    const int64_t cap = std::max<int64_t>(s->tab_cap, 1024);
    s->tab_cap = 0;
    pstd_status st = solver_ensure_tables(s, cap);
    if (st) return st;
    pulse_reset(s);  // the packet's table of step 0
    return PSTD_OK;
}

hipError_t pulse_launch_pre(const pstd_solver* s, int koff, const int* list, int64_t n_shell, float2* stage,
                            hipStream_t stream) {
    const PulseState* ps = s->pulse;
    if (!ps) return hipSuccess;
    if (stage && (koff < 0 || koff >= kStageSteps)) return hipErrorInvalidValue;
    const int table_blocks = ps->n_cells ? (ps->J + 3) / 4 : 0;
    const int source_blocks = koff >= 0 ? (int)((ps->n_cells + 255) / 256) : 0;
    const int stage_blocks = stage && koff >= 0 ? (int)((n_shell + 255) / 256) : 0;
    if (table_blocks + source_blocks + stage_blocks == 0) return hipSuccess;
    static_assert(kModeChunk == 256, "a table block computes one mode amplitude per thread");
    hipLaunchKernelGGL(pulse_pre_kernel, dim3((unsigned)(table_blocks + source_blocks + stage_blocks)), dim3(256), 0,
                       stream, s->ctr, koff, ps->K, ps->coef, ps->theta, ps->k_lo, ps->dk, ps->J, ps->ekd, ps->tab,
                       table_blocks, ps->n_cells, ps->cell, ps->j0, ps->w, ps->ab, source_blocks, s->buf[0],
                       s->buf[1], list, stage ? n_shell : 0, stage);
    return hipGetLastError();
}

namespace {

// the incident phasor at the grid origin (Eq. incpsiphasor) over the window
// steps run since the last reset, [max(dft_begin, from), min(dft_end,
// step)): per mode a geometric series in phi = W dtau - theta_l, taken whole
// so that it does not depend on how the steps were split into runs,
//   sum_{n=a}^{b-1} e^{i phi n} = e^{i phi (a + (m-1)/2)} sin(m phi / 2) / sin(phi / 2)
std::complex<double> incident_phasor(const pstd_solver* s, int f) {
    const PulseState* ps = s->pulse;
    const int64_t a = std::max(ps->from, s->prob.dft_begin), b = std::min(s->step, s->prob.dft_end);
    if (b <= a) return 0.0;
    const double m = (double)(b - a);
    std::complex<double> acc = 0;
    for (int l = 0; l < ps->K; ++l) {
        const double phi = ps->W[f] * s->dtau - ps->theta_h[l];
        const double sh = std::sin(0.5 * phi);
        const double ratio = std::fabs(sh) < 1e-300 ? m : std::sin(0.5 * m * phi) / sh;
        acc += std::complex<double>(ps->g[l].x, ps->g[l].y) * std::polar(ratio, phi * ((double)a + 0.5 * (m - 1)));
    }
    return acc;
}

}  // namespace

namespace {

// the packet's table of the current step (the device counter holds it), read
// by the step's first launch
hipError_t prime_table(pstd_solver* s) {
    hipError_t e = pulse_launch_pre(s, -1, nullptr, 0, nullptr, s->stream);
    return e == hipSuccess ? hipStreamSynchronize(s->stream) : e;
}

int64_t box_sum_bytes(const pstd_solver* s, int a) {
    return (int64_t)s->pulse->kbar.size() * 8 * s->points[a] * (int64_t)sizeof(double2);
}

}  // namespace

void pulse_reset(pstd_solver* s) {
    if (!s->pulse) return;
    s->pulse->from = s->step;
    (void)prime_table(s);
    for (int a = 0; a < 3; ++a)
        if (s->pulse->bacc[a]) (void)hipMemset(s->pulse->bacc[a], 0, box_sum_bytes(s, a));
}

int64_t pulse_state_bytes(const pstd_solver* s) {
    if (!s->pulse || !s->pulse->box) return 0;
    return box_sum_bytes(s, 0) + box_sum_bytes(s, 1) + box_sum_bytes(s, 2);
}

hipError_t pulse_save(const pstd_solver* s, char* dst, hipStream_t stream) {
    if (!s->pulse || !s->pulse->box) return hipSuccess;
    for (int a = 0; a < 3; ++a) {
        if (hipError_t e = hipMemcpyAsync(dst, s->pulse->bacc[a], box_sum_bytes(s, a), hipMemcpyDeviceToDevice, stream))
            return e;
        dst += box_sum_bytes(s, a);
    }
    return hipSuccess;
}

hipError_t pulse_load(pstd_solver* s, const char* src, int64_t from) {
    PulseState* ps = s->pulse;
    if (!ps) return hipSuccess;
    ps->from = from;
    if (ps->box)
        for (int a = 0; a < 3; ++a) {
            if (hipError_t e = hipMemcpyAsync(ps->bacc[a], src, box_sum_bytes(s, a), hipMemcpyDeviceToDevice, s->stream))
                return e;
            src += box_sum_bytes(s, a);
        }
    return prime_table(s);
}

float2* pulse_box_stage(const pstd_solver* s, int axis) { return s->pulse ? s->pulse->bstage[axis] : nullptr; }

hipError_t pulse_launch_box_flush(const pstd_solver* s, int count, hipStream_t stream) {
    const PulseState* ps = s->pulse;
    if (!ps || !ps->box) return hipSuccess;
    if (count < 1 || count > kStageSteps) return hipErrorInvalidValue;
    const int nk = (int)ps->kbar.size();
    BoxFlush bf{};
    int blocks = 0;
    for (int a = 0; a < 3; ++a) {
        bf.stage[a] = ps->bstage[a];
        bf.acc[a] = ps->bacc[a];
        bf.points[a] = s->points[a];
        bf.blocks[a] = (int)((nk * 4 * s->points[a] + 255) / 256);
        blocks += bf.blocks[a];
    }
    hipLaunchKernelGGL(box_flush_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, s->ctr, count, s->dft_tab,
                       s->w_tab, s->tab_cap, nk, bf);
    return hipGetLastError();
}

pstd_status pulse_box_output(pstd_solver* s, int ik, bool rescaled, BoxOut* o) {
    PulseState* ps = s->pulse;
    if (!ps || !ps->box) return solver_fail(s, PSTD_ESTATE, "no pulsed run on the box surface");
    if (ik < 0 || ik >= (int)ps->kbar.size()) return solver_fail(s, PSTD_EINVAL, "wavenumber index out of range");
    const std::complex<double> inc = incident_phasor(s, ik);
    const std::complex<double> inv = 1.0 / inc;
    if (!(std::abs(inc) > 0) || !std::isfinite(inv.real()) || !std::isfinite(inv.imag()))
        return solver_fail(s, PSTD_ESTATE, "the incident phasor of this wavenumber is zero");
    // the phasors of wavenumber k are those of the central wave in units
    // rescaled by k: k0 -> k k0, dxb -> k dxb, d/dxb -> (1/k) d/dxb
    const double k = rescaled ? ps->kbar[ik] : 1.0;
    o->prob = s->prob;
    o->prob.k0 = s->prob.k0 * k;
    for (int a = 0; a < 3; ++a) {
        o->dxb[a] = s->dxb[a] * k;
        o->acc[a] = ps->bacc[a] + (int64_t)ik * 8 * s->points[a];
    }
    const std::complex<double> d = inv / k;
    o->scale = PhasorScale{make_double2(inv.real(), inv.imag()), make_double2(d.real(), d.imag())};
    o->proj = &ps->proj[ik];
    return PSTD_OK;
}

pstd_status pulse_output(pstd_solver* s, int ik, SphereOut* o) {
    if (!s->pulse) {
        if (ik != 0) return solver_fail(s, PSTD_EINVAL, "without a pulse the only wavenumber index is 0");
        *o = SphereOut{0, make_double2(1.0 / s->inc_sum, 0.0), 1.0};
        return PSTD_OK;
    }
    PulseState* ps = s->pulse;
    if (ik < 0 || ik >= (int)ps->kbar.size()) return solver_fail(s, PSTD_EINVAL, "wavenumber index out of range");
    const std::complex<double> inc = incident_phasor(s, ik);
    const std::complex<double> inv = 1.0 / inc;
    if (!(std::abs(inc) > 0) || !std::isfinite(inv.real()) || !std::isfinite(inv.imag()))
        return solver_fail(s, PSTD_ESTATE, "the incident phasor of this wavenumber is zero");
    *o = SphereOut{ik, make_double2(inv.real(), inv.imag()), ps->kbar[ik]};
    return PSTD_OK;
}

}  // namespace pstd
