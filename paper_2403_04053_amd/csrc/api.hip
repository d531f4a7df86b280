// Host side of libpstd: validation, FP64 table construction, device state,
// the time-stepping loop (graph-replayed step groups) and the tile autotuner.
// See include/pstd.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "solver.hpp"

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kGraphSteps = 16;  // steps per replayed graph

thread_local std::string g_create_error;

// Device scratch of pstd_check_state_noalloc: the two FP64 norm reductions
// (result and per-workgroup partials of each).  One copy per device, held
// until the process ends; host code uses only the address each device
// reports for it (g_scratch_dev), never the array's name.
constexpr int kStaticScratchDoubles = 4096;  // 32 KiB
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];
std::mutex g_scratch_mu;                      // one user of the array at a time
double* g_scratch_dev[kMaxDevices] = {};      // its address on each device

// Look up the array's address on `device`, which must be current; once per device.
hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = static_cast<double*>(p);
    return hipSuccess;
}

pstd_status fail(pstd_solver* s, pstd_status st, const std::string& msg) {
    if (s) s->err = msg;
    else g_create_error = msg;
    return st;
}

pstd_status hip_fail(pstd_solver* s, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(s, e == hipErrorOutOfMemory ? PSTD_ENOMEM : PSTD_EHIP, m);
}

#define HIP_TRY(s, call)                                       \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return hip_fail((s), _e, #call); \
    } while (0)

double xi(double r) { return r - 2.0 / (3.0 * kPi) * std::sin(2 * kPi * r) + 1.0 / (12.0 * kPi) * std::sin(4 * kPi * r); }
double dxi(double r) { return 1.0 - 4.0 / 3.0 * std::cos(2 * kPi * r) + 1.0 / 3.0 * std::cos(4 * kPi * r); }
double d2xi(double r) { return 8.0 * kPi / 3.0 * std::sin(2 * kPi * r) - 4.0 * kPi / 3.0 * std::sin(4 * kPi * r); }

double ramp_of(double tau, double tau_r) {
    if (tau_r <= 0) return 1.0;
    double r = tau / tau_r;
    if (r < 0) r = 0;
    if (r > 1) r = 1;
    return xi(r);
}

double kbar_of(int m, int N, double dxb) {
    const int mp = m < N / 2 ? m : m - N;
    return 2.0 * kPi * mp / (N * dxb);
}

pstd_status reduced(const pstd_problem* p, double* E0, double* dxb, double* dtau, double* eta, double* dtau_crit) {
    *E0 = p->hbar * p->hbar * p->k0 * p->k0 / (2.0 * p->mass);
    double s = 0;
    for (int a = 0; a < 3; ++a) {
        dxb[a] = p->k0 * p->h[a];
        s += 1.0 / (dxb[a] * dxb[a]);
    }
    // largest |v|: the potential (inside the taper core) or the absorber's
    // real part (inside the layers; largest where the layers of all axes meet)
    int layers = 0;
    for (int a = 0; a < 3; ++a) layers += p->abc_cells[a] > 0;
    const double vmax = std::max(p->v_max / *E0, std::fabs(p->abc_UR) * layers);
    if (p->scheme == 1) {
        // FDTD: the stencil's symbol peaks at the Nyquist corner, |alpha_0 + 2 sum_l alpha_l (-1)^l|
        double sym = pstd::kFdtdAlpha[0];
        for (int l = 1; l <= 4; ++l) sym += 2.0 * pstd::kFdtdAlpha[l] * ((l & 1) ? -1.0 : 1.0);
        *dtau_crit = 1.0 / (std::fabs(sym) * s + vmax);
    } else {
        *dtau_crit = 1.0 / (kPi * kPi * s + vmax);
    }
    *dtau = p->dt > 0 ? *E0 * p->dt / p->hbar : 0.9 * *dtau_crit;
    *eta = std::sin(*dtau) / *dtau;
    return PSTD_OK;
}

pstd_status validate(const pstd_problem* p) {
    if (!p) return fail(nullptr, PSTD_EINVAL, "null problem");
    if (!(p->hbar > 0 && p->mass > 0 && p->k0 > 0)) return fail(nullptr, PSTD_EINVAL, "hbar, mass and k0 must be positive");
    if (!(p->v_max >= 0)) return fail(nullptr, PSTD_EINVAL, "v_max must be >= 0");
    if (!(p->dt >= 0)) return fail(nullptr, PSTD_EINVAL, "dt must be >= 0");
    if (!std::isfinite(p->abc_UR) || !(p->abc_alphaR >= 0))
        return fail(nullptr, PSTD_EINVAL, "abc_UR must be finite and abc_alphaR >= 0");
    if (p->scheme != 0 && p->scheme != 1) return fail(nullptr, PSTD_EINVAL, "scheme must be 0 or 1");
    if (p->scheme == 1) {
        if (p->sub_core[0] || p->sub_core[1] || p->sub_core[2])
            return fail(nullptr, PSTD_EUNSUPPORTED, "the FDTD scheme has no subdomain mode");
        if (p->surface_kind == 0 && p->dft_end > p->dft_begin)
            return fail(nullptr, PSTD_EUNSUPPORTED,
                        "the FDTD scheme accumulates the surface DFT on the spherical surface only (surface_kind 1)");
    }
    for (int a = 0; a < 3; ++a) {
        const int N = p->n[a];
        if (N < 8 || (N & 1)) return fail(nullptr, PSTD_EINVAL, "grid lengths must be even and >= 8");
        if (!(p->h[a] > 0)) return fail(nullptr, PSTD_EINVAL, "grid spacing must be positive");
        if (p->scheme == 1) {
            // the stencil works on any length
        } else if (p->sub_core[a] > 0) {
            const int C = p->sub_core[a], nloc = C + 2 * p->sub_halo;
            if (N % C) return fail(nullptr, PSTD_EINVAL, "sub_core must divide the grid length");
            if (p->sub_taper < 0 || p->sub_halo < p->sub_taper + 5)
                return fail(nullptr, PSTD_EINVAL, "sub_halo must be at least sub_taper + 5 (Section 2.6)");
            int v;
            if (pstd::pass_variants(nloc, true, &v, 1) == 0)
                return fail(nullptr, PSTD_EUNSUPPORTED, "no FFT pass compiled for local length " + std::to_string(nloc));
        } else if (p->sub_core[a] < 0) {
            return fail(nullptr, PSTD_EINVAL, "sub_core must be >= 0");
        } else if (int v; pstd::pass_variants(N, false, &v, 1) == 0) {
            return fail(nullptr, PSTD_EUNSUPPORTED, "no FFT pass compiled for axis length " + std::to_string(N));
        }
        const int* y = p->tfsf[a];
        if (!(0 <= y[0] && y[0] < y[1] && y[1] <= y[2] && y[2] < y[3] && y[3] <= N - 1))
            return fail(nullptr, PSTD_EINVAL, "taper indices must satisfy 0 <= y0 < y1 <= y2 < y3 <= N-1");
        if (p->abc_cells[a] < 0 || 2 * p->abc_cells[a] > N) return fail(nullptr, PSTD_EINVAL, "absorber wider than the grid");
        const int lo = p->surf_lo[a], hi = p->surf_hi[a];
        if (!(0 <= lo && lo < hi && hi <= N - 1)) return fail(nullptr, PSTD_EINVAL, "box faces out of range");
        if (!(lo <= y[0] && hi >= y[3]))
            return fail(nullptr, PSTD_EINVAL, "box faces must lie wholly in the scattered-field region (face <= y0, >= y3)");
        if (lo < p->abc_cells[a] || N - 1 - hi < p->abc_cells[a])
            return fail(nullptr, PSTD_EINVAL, "box faces must lie outside the absorbing layer");
    }
    if (p->dft_begin < 0 || p->dft_end < p->dft_begin) return fail(nullptr, PSTD_EINVAL, "bad DFT window");
    return PSTD_OK;
}

// Real part of the complex absorbing potential along axis a (units of E0):
// abc_UR / cosh^2(alpha d) inside the layer, the shape of the mask's rate
std::vector<double> absorber_real(const pstd_problem& p, int a) {
    const int N = p.n[a], P = p.abc_cells[a];
    const double al = p.abc_alphaR > 0 ? p.abc_alphaR : p.abc_alpha;
    std::vector<double> w(N, 0.0);
    if (p.abc_UR == 0.0) return w;
    for (int i = 0; i < N; ++i) {
        const int d = std::min(i, N - 1 - i);
        if (d < P) {
            const double c = std::cosh(al * d);
            w[i] = p.abc_UR / (c * c);
        }
    }
    return w;
}

// The box where V may be non-zero: the taper's core y1 <= i <= y2 per axis
// (Section 2.2.2: (zeta - 1) V = 0)
void potential_box(const pstd_problem& p, int lo[3], int n[3]) {
    for (int a = 0; a < 3; ++a) {
        lo[a] = p.tfsf[a][1];
        n[a] = p.tfsf[a][2] - p.tfsf[a][1] + 1;
    }
}

// 2 dtau V / E0 on that box, [z][y][x]; V in energy units over the whole
// grid (null: V = 0)
std::vector<float> scaled_potential(const pstd_solver* s, const float* V) {
    const pstd_problem& p = s->prob;
    int lo[3], n[3];
    potential_box(p, lo, n);
    const double scale = 2.0 * s->dtau / s->E0;
    std::vector<float> box((size_t)n[0] * n[1] * n[2], 0.0f);
    if (!V) return box;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                const int64_t id = (i + lo[0]) + (int64_t)p.n[0] * ((j + lo[1]) + (int64_t)p.n[1] * (k + lo[2]));
                box[i + (size_t)n[0] * (j + (size_t)n[1] * k)] = (float)(scale * (double)V[id]);
            }
    return box;
}

// 2 dtau (V / E0 + sum_a w_a) on every cell, [k][j][i] (the FDTD scheme's
// potential array; null V: the absorber's real part alone)
std::vector<float> scaled_potential_full(const pstd_solver* s, const float* V) {
    const pstd_problem& p = s->prob;
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const std::vector<double> wx = absorber_real(p, 0), wy = absorber_real(p, 1), wz = absorber_real(p, 2);
    const double scale = 2.0 * s->dtau / s->E0, sw = 2.0 * s->dtau;
    std::vector<float> v2((size_t)s->cells);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t id = i + (int64_t)nx * (j + (int64_t)ny * k);
                const double v = V ? (double)V[id] : 0.0;
                v2[id] = (float)(scale * v + sw * (wx[i] + wy[j] + wz[k]));
            }
    return v2;
}

template <class T>
pstd_status upload(pstd_solver* s, T* dst, const std::vector<T>& src) {
    HIP_TRY(s, hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return PSTD_OK;
}

// local spectral length of axis a (the subdomain length in the segmented mode)
int local_len(const pstd_problem& p, int a) {
    return p.sub_core[a] > 0 ? p.sub_core[a] + 2 * p.sub_halo : p.n[a];
}

// plane index of side `side` along axis a as (segment, position in the local array)
void plane_local(const pstd_problem& p, int a, int side, int* seg, int* pos) {
    const int i0 = side == 0 ? p.surf_lo[a] : p.surf_hi[a];
    if (p.sub_core[a] > 0) {
        *seg = i0 / p.sub_core[a];
        *pos = i0 - *seg * p.sub_core[a] + p.sub_halo;
    } else {
        *seg = 0;
        *pos = i0;
    }
}

// taper factor of axis a at grid index i and its derivatives in reduced
// length (Eq. zeta_y with Eq. xi)
void taper(const pstd_problem& p, int a, double dxb, int i, double* z, double* z1, double* z2) {
    const int* y = p.tfsf[a];
    *z = 0;
    *z1 = 0;
    *z2 = 0;
    if (i > y[0] && i < y[3]) {
        if (i >= y[1] && i <= y[2]) {
            *z = 1.0;
        } else if (i < y[1]) {
            const double w = (y[1] - y[0]) * dxb, r = double(i - y[0]) / (y[1] - y[0]);
            *z = xi(r);
            *z1 = dxi(r) / w;
            *z2 = d2xi(r) / (w * w);
        } else {
            const double w = (y[3] - y[2]) * dxb, r = double(i - y[2]) / (y[3] - y[2]);
            *z = 1.0 - xi(r);
            *z1 = -dxi(r) / w;
            *z2 = -d2xi(r) / (w * w);
        }
    }
}

pstd_status build_tables(pstd_solver* s) {
    const pstd_problem& p = s->prob;
    // per axis: kk[Nl] f, wloc[Nl] f, tw[Nl] f2, dlo[Nl] f2, dhi[Nl] f2 (local length Nl),
    //           gam[N] f, zt[N] f2, dz[N] f2, zd[N] f4 (global length N)
    size_t bytes = 0;
    for (int a = 0; a < 3; ++a)
        bytes += (size_t)local_len(p, a) * (2 * sizeof(float) + 3 * sizeof(float2)) +
                 (size_t)p.n[a] * (sizeof(float) + 2 * sizeof(float2) + sizeof(float4)) + 16 * 9;
    HIP_TRY(s, hipMalloc(&s->tables, bytes));
    char* cur = (char*)s->tables;
    for (int a = 0; a < 3; ++a) {
        const int N = p.n[a];
        const int Nl = local_len(p, a);
        const double dxb = s->dxb[a];
        std::vector<float> kk(Nl), wl(Nl, 1.0f), gam(N);
        std::vector<float2> tw(Nl), zt(N), dz(N), dlo(Nl), dhi(Nl);
        for (int m = 0; m < Nl; ++m) {
            const double k = kbar_of(m, Nl, dxb);
            kk[m] = (float)(2.0 * s->eta * s->dtau * k * k / Nl);
            tw[m] = make_float2((float)std::cos(2 * kPi * m / Nl), (float)-std::sin(2 * kPi * m / Nl));
        }
        if (p.sub_core[a] > 0) {
            // halo weights, distal to proximal (Eq. weight): 0, xi(l/(n_t+1)) for l = 1..n_t, then 1
            const int H = p.sub_halo, nt = p.sub_taper;
            for (int l = 0; l < H; ++l) {
                const double w = l == 0 ? 0.0 : (l <= nt ? xi(double(l) / (nt + 1)) : 1.0);
                wl[l] = (float)w;
                wl[Nl - 1 - l] = (float)w;
            }
        }
        for (int i = 0; i < N; ++i) {
            const int d = std::min(i, N - 1 - i);
            double g = 0.0;
            if (d < p.abc_cells[a]) {
                const double c = std::cosh(p.abc_alpha * d);
                g = p.abc_U0 / (c * c);
            }
            gam[i] = (float)std::exp(-g * s->dtau);
            double z, z1, z2;
            taper(p, a, dxb, i, &z, &z1, &z2);
            const double x = (i - N / 2) * dxb;
            const double ph = s->kh[a] * x;
            const double er = std::cos(ph), ei = std::sin(ph);
            zt[i] = make_float2((float)(z * er), (float)(z * ei));
            // (z2 + 2 i kh z1) e^{i ph}
            const double ar = z2, ai = 2.0 * s->kh[a] * z1;
            dz[i] = make_float2((float)(ar * er - ai * ei), (float)(ar * ei + ai * er));
            if (p.scheme == 1) {
                // sharp box T = [y1 <= i <= y2]; zt = T e^{i ph}, dz = -C e^{i ph} / dxb^2 with
                // C = sum_l alpha_l sum_pm [T(i) - T(i pm l)] e^{pm i kh l dxb} (wall terms)
                const int* y = p.tfsf[a];
                auto T = [&](int j) { return (j >= y[1] && j <= y[2]) ? 1.0 : 0.0; };
                double cr = 0, ci = 0;
                for (int l = 1; l <= 4; ++l)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        const double w = pstd::kFdtdAlpha[l] * (T(i) - T(i + sg * l));
                        cr += w * std::cos(sg * s->kh[a] * l * dxb);
                        ci += w * std::sin(sg * s->kh[a] * l * dxb);
                    }
                const double f = -1.0 / (dxb * dxb);
                zt[i] = make_float2((float)(T(i) * er), (float)(T(i) * ei));
                dz[i] = make_float2((float)(f * (cr * er - ci * ei)), (float)(f * (cr * ei + ci * er)));
            }
        }
        // spectral-derivative rows: d(e) = (1/Nl) sum_m i kbar_m exp(2 pi i m (i0 - e)/Nl)
        for (int side = 0; side < 2; ++side) {
            int seg, i0;
            plane_local(p, a, side, &seg, &i0);
            std::vector<float2>& row = side == 0 ? dlo : dhi;
            for (int e = 0; e < Nl; ++e) {
                double re = 0, im = 0;
                for (int m = 0; m < Nl; ++m) {
                    const double k = kbar_of(m, Nl, dxb);
                    const double ang = 2 * kPi * (double)(((int64_t)m * (i0 - e)) % Nl) / Nl;
                    // i k e^{i ang}
                    re += -k * std::sin(ang);
                    im += k * std::cos(ang);
                }
                row[e] = make_float2((float)(re / Nl), (float)(im / Nl));
            }
        }
        auto place = [&](auto& vec) {
            using T = typename std::decay_t<decltype(vec)>::value_type;
            T* ptr = (T*)cur;
            cur += ((vec.size() * sizeof(T) + 15) / 16) * 16;
            return ptr;
        };
        float* d_kk = place(kk);
        float* d_wl = place(wl);
        float* d_gam = place(gam);
        float2* d_tw = place(tw);
        float2* d_zt = place(zt);
        float2* d_dz = place(dz);
        std::vector<float4> zd(N);
        for (int i = 0; i < N; ++i) zd[i] = make_float4(zt[i].x, zt[i].y, dz[i].x, dz[i].y);
        float4* d_zd = place(zd);
        float2* d_dlo = place(dlo);
        float2* d_dhi = place(dhi);
        pstd_status st;
        if ((st = upload(s, d_kk, kk)) || (st = upload(s, d_wl, wl)) || (st = upload(s, d_gam, gam)) ||
            (st = upload(s, d_tw, tw)) || (st = upload(s, d_zt, zt)) || (st = upload(s, d_dz, dz)) ||
            (st = upload(s, d_zd, zd)) || (st = upload(s, d_dlo, dlo)) || (st = upload(s, d_dhi, dhi)))
            return st;
        s->ax[a] = pstd::AxisTables{d_kk, d_tw, d_gam, d_zt, d_dz, d_zd, d_dlo, d_dhi};
        s->wloc[a] = d_wl;
    }
    return PSTD_OK;
}


// ---------------------------------------------------------------------------
// per-step launches
// ---------------------------------------------------------------------------

// launch step ctr[0] + koff, step koff of a group of `count` launched
// together, on `stream`
// the FDTD step's arguments (scheme 1)
pstd::FdtdArgs fdtd_args(const pstd_solver* s) {
    pstd::FdtdArgs a{};
    a.buf[0] = s->buf[0];
    a.buf[1] = s->buf[1];
    a.v2 = s->v2full;
    a.nx = s->prob.n[0];
    a.ny = s->prob.n[1];
    a.nz = s->prob.n[2];
    double kc = 0;
    for (int ax = 0; ax < 3; ++ax) {
        a.gam[ax] = s->ax[ax].gam;
        a.zt[ax] = s->ax[ax].zt;
        a.dz[ax] = s->ax[ax].dz;
        const double f = -2.0 * s->dtau / (s->dxb[ax] * s->dxb[ax]);
        kc += f * pstd::kFdtdAlpha[0];
        for (int l = 1; l <= 4; ++l) a.k[ax][l - 1] = (float)(f * pstd::kFdtdAlpha[l]);
    }
    a.kc = (float)kc;
    a.ctr = s->ctr;
    a.sigma_tab = s->sigma_tab;
    return a;
}

pstd_status launch_passes(pstd_solver* s, hipStream_t stream, int koff, int count, hipEvent_t* ev) {
    if (s->pulse) {
        // the packet's table of the next step, this step's layer source (into
        // psi^{n-1}, before the z pass), and psi^n on the shell into the
        // group's ring (added at the group's end), in one launch
        const int* list;
        int64_t n_shell;
        float2* stage;
        pstd::sphere_stage_buffers(s, &list, &n_shell, &stage);
        hipError_t e = pstd::pulse_launch_pre(s, koff, list, n_shell, stage, stream);
        if (e != hipSuccess) return hip_fail(s, e, "pulse table / shell stage launch");
    } else if (pstd::sphere_staged(s)) {
        hipError_t e = pstd::sphere_launch_stage(s, koff, stream);
        if (e != hipSuccess) return hip_fail(s, e, "shell stage launch");
    } else if (s->sphere) {
        // shell DFT in pairs of steps of the group (the odd step adds the even
        // one before it; a last even step goes alone), before this step
        // overwrites psi^{n-1}
        const int k = (koff & 1) ? 2 : (koff == count - 1 ? 1 : 0);
        hipError_t e = pstd::sphere_launch_dft(s, koff, k, stream);
        if (e != hipSuccess) return hip_fail(s, e, "shell DFT launch");
    }
    if (s->prob.scheme == 1) {
        // one stencil kernel per step; its time goes to the x slot of the timers
        if (ev) HIP_TRY(s, hipEventRecord(ev[0], stream));
        hipError_t e = pstd::launch_fdtd(fdtd_args(s), koff, stream);
        if (e != hipSuccess) return hip_fail(s, e, "FDTD launch");
        if (ev)
            for (int i = 1; i < 6; ++i) HIP_TRY(s, hipEventRecord(ev[i], stream));
        return PSTD_OK;
    }
    for (int axis = 0; axis < 3; ++axis) {
        pstd::PassArgs a;
        pstd::solver_args(s, axis, a);
        const bool seg = s->prob.sub_core[axis] > 0;
        if (ev) HIP_TRY(s, hipEventRecord(ev[2 * axis], stream));
        hipError_t e = pstd::launch_variant_single(s->variant[axis], seg, axis, a, koff, stream);
        if (e != hipSuccess) return hip_fail(s, e, "pass launch");
        if (ev) HIP_TRY(s, hipEventRecord(ev[2 * axis + 1], stream));
    }
    if (s->pulse && koff == count - 1) {
        // a pulsed run on the box: the group's staged plane values into the sums
        hipError_t e = pstd::pulse_launch_box_flush(s, count, stream);
        if (e != hipSuccess) return hip_fail(s, e, "plane flush launch");
    }
    if (pstd::sphere_staged(s) && koff == count - 1) {
        // the group's staged steps into the phasor sums (before the counter advances)
        hipError_t e = pstd::sphere_launch_flush(s, count, stream);
        if (e != hipSuccess) return hip_fail(s, e, "shell flush launch");
    }
    return PSTD_OK;
}

// `count` consecutive steps, then one counter advance
pstd_status launch_steps(pstd_solver* s, hipStream_t stream, int count, hipEvent_t* ev) {
    for (int k = 0; k < count; ++k) {
        pstd_status st = launch_passes(s, stream, k, count, ev);
        if (st) return st;
    }
    hipError_t e = pstd::launch_advance(s->ctr, 1, count, stream);
    if (e != hipSuccess) return hip_fail(s, e, "advance launch");
    return PSTD_OK;
}

pstd_status build_graph(pstd_solver* s) {
    if (s->graph) return PSTD_OK;
    if (!s->cap_stream) HIP_TRY(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    HIP_TRY(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    pstd_status st = launch_steps(s, s->cap_stream, kGraphSteps, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(s, e, "graph capture");
    e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        s->graph = nullptr;
        return hip_fail(s, e, "graph instantiate");
    }
    return PSTD_OK;
}

}  // namespace

namespace pstd {

pstd_status solver_fail(pstd_solver* s, pstd_status st, const std::string& msg) { return fail(s, st, msg); }

void solver_taper(const pstd_problem& p, int a, double dxb, int i, double* z, double* z1, double* z2) {
    taper(p, a, dxb, i, z, z1, z2);
}

void solver_incident_axis(const pstd_solver* s, int a, std::vector<double2>& out) {
    const int N = s->prob.n[a];
    out.resize(N);
    const int* y = s->prob.tfsf[a];
    for (int i = 0; i < N; ++i) {
        double z, z1, z2;
        taper(s->prob, a, s->dxb[a], i, &z, &z1, &z2);
        // the FDTD scheme's total-field region is the sharp box y1 <= i <= y2
        if (s->prob.scheme == 1) z = (i >= y[1] && i <= y[2]) ? 1.0 : 0.0;
        const double ph = s->kh[a] * (i - N / 2) * s->dxb[a];
        out[i] = make_double2(z * std::cos(ph), z * std::sin(ph));
    }
}
pstd_status solver_hip_fail(pstd_solver* s, hipError_t e, const char* what) { return hip_fail(s, e, what); }

void solver_args(const pstd_solver* s, int axis, PassArgs& a) {
    a = PassArgs{};
    const pstd_problem& p = s->prob;
    a.buf[0] = s->buf[0];
    a.buf[1] = s->buf[1];
    a.L = s->L;
    a.pot = s->pot;
    a.potx = s->potx;
    a.nt = s->nt;
    a.nx = p.n[0];
    a.ny = p.n[1];
    a.nz = p.n[2];
    for (int i = 0; i < 3; ++i) a.ax[i] = s->ax[i];
    a.ctr = s->ctr;
    a.sigma_tab = s->sigma_tab;
    a.w_tab = s->w_tab;
    a.dft_tab = s->dft_zero ? s->dft_zero : s->dft_tab;
    plane_local(p, axis, 0, &a.seg_plane[0], &a.plane_lo);
    plane_local(p, axis, 1, &a.seg_plane[1], &a.plane_hi);
    a.acc = s->acc[axis];
    a.points = s->points[axis];
    const bool seg = p.sub_core[axis] > 0;
    a.seg_core = seg ? p.sub_core[axis] : 0;
    a.seg_halo = seg ? p.sub_halo : 0;
    a.nseg = seg ? p.n[axis] / p.sub_core[axis] : 1;
    a.wloc = s->wloc[axis];
    a.bstage = pulse_box_stage(s, axis);
    variant_tiles(s->variant[axis], axis, a);
}

pstd_status solver_ensure_tables(pstd_solver* s, int64_t n_end) {
    if (n_end <= s->tab_cap) return PSTD_OK;
    int64_t cap = std::max<int64_t>(n_end, 2 * s->tab_cap);
    cap = std::max<int64_t>(cap, 1024);
    // one row of DFT weights per wavenumber (several with a pulse, whose
    // source comes from its own kernels: sigma = 0)
    const int nk = pulse_wavenumbers(s);
    std::vector<float2> sig(cap);
    std::vector<double2> w(nk * cap);
    std::vector<int> on(cap);
    const double fac = 2.0 * s->dtau * (s->prob.eta_on_source && s->prob.scheme == 0 ? s->eta : 1.0);
    for (int64_t n = 0; n < cap; ++n) {
        const double tau = n * s->dtau;
        const double f = fac * ramp_of(tau, s->tau_r);
        const double ph = s->omega * tau;
        sig[n] = s->pulse ? make_float2(0.f, 0.f) : make_float2((float)(f * std::cos(ph)), (float)(-f * std::sin(ph)));
        // the DFT at the incident wave's frequency (1, the FDTD scheme's W,
        // or each wavenumber's frequency of a pulse)
        for (int k = 0; k < nk; ++k) {
            const double om = pulse_frequency(s, k) * tau;
            w[k * cap + n] = make_double2(std::cos(om), std::sin(om));
        }
        on[n] = (n >= s->prob.dft_begin && n < s->prob.dft_end) ? 1 : 0;
    }
    // queued steps may still read the old tables
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    (void)hipFree(s->sigma_tab);
    (void)hipFree(s->w_tab);
    (void)hipFree(s->dft_tab);
    (void)hipFree(s->dft_zero);
    s->sigma_tab = nullptr;
    s->w_tab = nullptr;
    s->dft_tab = nullptr;
    s->dft_zero = nullptr;
    s->tab_cap = 0;
    HIP_TRY(s, hipMalloc(&s->sigma_tab, cap * sizeof(float2)));
    HIP_TRY(s, hipMalloc(&s->w_tab, nk * cap * sizeof(double2)));
    HIP_TRY(s, hipMalloc(&s->dft_tab, cap * sizeof(int)));
    HIP_TRY(s, hipMemcpy(s->sigma_tab, sig.data(), cap * sizeof(float2), hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemcpy(s->w_tab, w.data(), nk * cap * sizeof(double2), hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemcpy(s->dft_tab, on.data(), cap * sizeof(int), hipMemcpyHostToDevice));
    if (s->prob.surface_kind == 1) {
        HIP_TRY(s, hipMalloc(&s->dft_zero, cap * sizeof(int)));
        HIP_TRY(s, hipMemset(s->dft_zero, 0, cap * sizeof(int)));
    }
    s->tab_cap = cap;
    s->tab_gen += 1;
    solver_drop_graph(s);  // the graph's launches hold the old table addresses
    return PSTD_OK;
}

void solver_account_steps(pstd_solver* s, int64_t from, int64_t to) {
    for (int64_t n = std::max(from, s->prob.dft_begin); n < std::min(to, s->prob.dft_end); ++n) {
        s->inc_sum += ramp_of(n * s->dtau, s->tau_r);
        s->win_steps += 1;
    }
}

void solver_drop_graph(pstd_solver* s) {
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
}

pstd_status solver_create(const pstd_problem* p, hipStream_t stream, int64_t* ext_ctr, pstd_solver** out) {
    *out = nullptr;
    pstd_status st = validate(p);
    if (st) return st;
    pstd_solver* s = new pstd_solver();
    s->prob = *p;
    s->stream = stream;
    (void)hipGetDevice(&s->device);
    double crit;
    reduced(p, &s->E0, s->dxb, &s->dtau, &s->eta, &crit);
    if (s->dtau > crit * (1 + 1e-12) && !p->force_dt) {
        delete s;
        return fail(nullptr, PSTD_EUNSTABLE, "dt exceeds the bound of Eq. PSTDstability");
    }
    const double th = p->theta, ph = p->phi;
    s->kh[0] = std::sin(th) * std::cos(ph);
    s->kh[1] = std::sin(th) * std::sin(ph);
    s->kh[2] = std::cos(th);
    if (p->scheme == 1) {
        // the walls drive the incident wave at the scheme's discrete frequency
        // for k_hat: sin(W dtau) = dtau k_h^2, k_h^2 = -sum_a symbol(kh_a dxb_a) / dxb_a^2
        double k2 = 0;
        for (int a = 0; a < 3; ++a) {
            const double th_a = s->kh[a] * s->dxb[a];
            double sym = pstd::kFdtdAlpha[0];
            for (int l = 1; l <= 4; ++l) sym += 2.0 * pstd::kFdtdAlpha[l] * std::cos(l * th_a);
            k2 -= sym / (s->dxb[a] * s->dxb[a]);
        }
        s->omega = std::asin(s->dtau * k2) / s->dtau;
    }
    s->tau_r = 2 * kPi * p->ramp_periods;
    s->cells = (int64_t)p->n[0] * p->n[1] * p->n[2];
    s->points[0] = (int64_t)p->n[1] * p->n[2];
    s->points[1] = (int64_t)p->n[0] * p->n[2];
    s->points[2] = (int64_t)p->n[0] * p->n[1];
    auto cleanup = [&](pstd_status e) {
        std::string m = s->err;
        pstd_destroy(s);
        g_create_error = m;
        return e;
    };
    hipError_t e;
    // the first device call: set-up of this device's static scratch
    if ((e = static_scratch_init(s->device))) return cleanup(hip_fail(s, e, "static scratch address"));
    if ((e = hipMalloc(&s->buf[0], s->cells * sizeof(float2))) || (e = hipMalloc(&s->buf[1], s->cells * sizeof(float2))) ||
        (e = hipMalloc(&s->L, s->cells * sizeof(float2))))
        return cleanup(hip_fail(s, e, "hipMalloc state"));
    if (ext_ctr) {
        s->ctr = ext_ctr;
        s->owns_ctr = false;
        s->in_batch = true;
    } else if ((e = hipMalloc(&s->ctr, 2 * sizeof(int64_t)))) {
        return cleanup(hip_fail(s, e, "hipMalloc counters"));
    }
    for (int a = 0; a < 3; ++a)
        if ((e = hipMalloc(&s->acc[a], 8 * s->points[a] * sizeof(double2)))) return cleanup(hip_fail(s, e, "hipMalloc acc"));
    for (int a = 0; a < 3; ++a) pass_variants(local_len(*p, a), p->sub_core[a] > 0, &s->variant[a], 1);
    if ((st = build_tables(s))) return cleanup(st);
    if (ext_ctr && p->surface_kind != 0)
        return cleanup(fail(s, PSTD_EUNSUPPORTED, "batch instances integrate over the box surface only"));
    if (ext_ctr && p->scheme != 0)
        return cleanup(fail(s, PSTD_EUNSUPPORTED, "batch instances run the spectral scheme only"));
    if ((st = sphere_create(s))) return cleanup(st);
    const int64_t c0[2] = {0, std::numeric_limits<int64_t>::max()};
    if ((e = hipMemcpy(s->ctr, c0, sizeof(c0), hipMemcpyHostToDevice))) return cleanup(hip_fail(s, e, "counters"));
    if ((e = hipMemset(s->buf[0], 0, s->cells * sizeof(float2))) || (e = hipMemset(s->buf[1], 0, s->cells * sizeof(float2))))
        return cleanup(hip_fail(s, e, "hipMemset"));
    // the potential term: V on the taper's core (zero until set), and the
    // complex absorber's real part as one table per axis
    potential_box(*p, s->pot.lo, s->pot.n);
    const int64_t nbox = (int64_t)s->pot.n[0] * s->pot.n[1] * s->pot.n[2];
    if ((e = hipMalloc(&s->vbox, nbox * sizeof(float))) || (e = hipMemset(s->vbox, 0, nbox * sizeof(float))))
        return cleanup(hip_fail(s, e, "potential"));
    s->pot.box = s->vbox;
    if (p->scheme == 1) {
        const std::vector<float> full = scaled_potential_full(s, nullptr);
        if ((e = hipMalloc(&s->v2full, full.size() * sizeof(float))) ||
            (e = hipMemcpy(s->v2full, full.data(), full.size() * sizeof(float), hipMemcpyHostToDevice)))
            return cleanup(hip_fail(s, e, "potential"));
    }
    // where the potential term is taken: in the x pass (re-reading psi^n from
    // the cache on the rows that cross V's box) when the box covers under a
    // quarter of the rows, else in the z pass (psi^n held in registers); the
    // complex absorber's real part (every cell) and segmented x pencils take
    // the z pass (batch instances follow the same rule, grouped by it)
    const double box_rows = (double)s->pot.n[1] * s->pot.n[2] / ((double)p->n[1] * p->n[2]);
    s->potx = (p->abc_UR == 0.0 && p->sub_core[0] == 0 && box_rows < 0.25) ? 1 : 0;
    // fields (psi pair and L, 24 B per cell) beyond the Infinity Cache: the z
    // pass's last-use loads bypass it, which leaves it to the lines the next
    // pass reads (measured: 256^3 +6 %, 288^3 +1 %; within the cache the
    // same hint costs 15-20 %)
    s->nt = 24.0 * (double)p->n[0] * p->n[1] * p->n[2] > kInfinityCacheBytes ? 1 : 0;
    if (p->abc_UR != 0.0) {
        std::vector<float> wr;
        for (int a = 0; a < 3; ++a)
            for (double w : absorber_real(*p, a)) wr.push_back((float)(2.0 * s->dtau * w));
        if ((e = hipMalloc(&s->wr, wr.size() * sizeof(float))) ||
            (e = hipMemcpy(s->wr, wr.data(), wr.size() * sizeof(float), hipMemcpyHostToDevice)))
            return cleanup(hip_fail(s, e, "absorber tables"));
        s->pot.wr[0] = s->wr;
        s->pot.wr[1] = s->wr + p->n[0];
        s->pot.wr[2] = s->wr + p->n[0] + p->n[1];
    }
    for (int a = 0; a < 3; ++a)
        if ((e = hipMemset(s->acc[a], 0, 8 * s->points[a] * sizeof(double2)))) return cleanup(hip_fail(s, e, "hipMemset acc"));
    // per-step tables through the end of the DFT window (up to 2^18 steps),
    // so a run of that length never reallocates them (and re-captures the graph)
    const int64_t tab_steps = std::min<int64_t>(std::max<int64_t>(p->dft_end, 1024), int64_t(1) << 18);
    if ((st = solver_ensure_tables(s, tab_steps))) return cleanup(st);
    if ((e = hipDeviceSynchronize())) return cleanup(hip_fail(s, e, "sync"));
    *out = s;
    return PSTD_OK;
}

// Time `reps` back-to-back launches of each given tile shape of one axis on
// scratch state of the solver's size (the solver's own state is untouched);
// ms_out[k] receives the average milliseconds per launch of shape ids[k].
pstd_status time_shapes(pstd_solver* s, int axis, const int* ids, int n, int32_t reps, float* ms_out) {
    float2 *tb0 = nullptr, *tb1 = nullptr, *tL = nullptr;
    double2* tacc = nullptr;
    int64_t* tctr = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        (void)hipFree(tb0);
        (void)hipFree(tb1);
        (void)hipFree(tL);
        (void)hipFree(tacc);
        (void)hipFree(tctr);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e;
    if ((e = hipMalloc(&tb0, s->cells * sizeof(float2))) || (e = hipMalloc(&tb1, s->cells * sizeof(float2))) ||
        (e = hipMalloc(&tL, s->cells * sizeof(float2))) || (e = hipMalloc(&tctr, 2 * sizeof(int64_t))) ||
        (e = hipMalloc(&tacc, 8 * s->points[axis] * sizeof(double2))) || (e = hipEventCreate(&e0)) ||
        (e = hipEventCreate(&e1)) || (e = hipMemset(tb0, 0, s->cells * sizeof(float2))) ||
        (e = hipMemset(tb1, 0, s->cells * sizeof(float2))) ||
        (e = hipMemset(tacc, 0, 8 * s->points[axis] * sizeof(double2)))) {
        release();
        return hip_fail(s, e, "timing scratch");
    }
    // a step inside the DFT window: the slower form of every pass
    int64_t win = s->prob.dft_end > s->prob.dft_begin ? s->prob.dft_begin : 0;
    if (win >= s->tab_cap) win = 0;
    const int64_t c0[2] = {win, std::numeric_limits<int64_t>::max()};
    if ((e = hipMemcpy(tctr, c0, sizeof(c0), hipMemcpyHostToDevice))) {
        release();
        return hip_fail(s, e, "timing scratch");
    }
    if (s->prob.scheme == 1) {
        // the FDTD step is one kernel: time it (whatever the axis or shape)
        FdtdArgs a = fdtd_args(s);
        a.buf[0] = tb0;
        a.buf[1] = tb1;
        a.ctr = tctr;
        float ms = 0;
        e = launch_fdtd(a, 0, s->stream);
        if (!e) e = hipEventRecord(e0, s->stream);
        for (int r = 0; r < reps && !e; ++r) e = launch_fdtd(a, 0, s->stream);
        if (!e) e = hipEventRecord(e1, s->stream);
        if (!e) e = hipEventSynchronize(e1);
        if (!e) e = hipEventElapsedTime(&ms, e0, e1);
        for (int k = 0; k < n; ++k) ms_out[k] = ms / reps;
        release();
        if (e) return hip_fail(s, e, "FDTD timing");
        return PSTD_OK;
    }
    const bool seg = s->prob.sub_core[axis] > 0;
    // two rounds over the candidates, the faster of each candidate's two
    // timings: the first candidates of a round may run before the clocks have
    // settled
    for (int k = 0; k < n; ++k) ms_out[k] = std::numeric_limits<float>::max();
    for (int round = 0; round < 2; ++round)
    for (int k = 0; k < n && !e; ++k) {
        PassArgs a;
        const int keep = s->variant[axis];
        s->variant[axis] = ids[k];
        solver_args(s, axis, a);
        s->variant[axis] = keep;
        a.buf[0] = tb0;
        a.buf[1] = tb1;
        a.L = tL;
        a.acc = tacc;
        a.ctr = tctr;
        float ms = 0;
        e = launch_variant_single(ids[k], seg, axis, a, 0, s->stream);
        if (!e) e = hipEventRecord(e0, s->stream);
        for (int r = 0; r < reps && !e; ++r) e = launch_variant_single(ids[k], seg, axis, a, 0, s->stream);
        if (!e) e = hipEventRecord(e1, s->stream);
        if (!e) e = hipEventSynchronize(e1);
        if (!e) e = hipEventElapsedTime(&ms, e0, e1);
        ms_out[k] = std::min(ms_out[k], ms / reps);
    }
    release();
    if (e) return hip_fail(s, e, "pass timing");
    return PSTD_OK;
}

pstd_status solver_autotune(pstd_solver* s, int32_t reps) {
    // time every compiled tile shape of each axis and keep the fastest (the
    // FDTD step has one shape)
    if (s->prob.scheme == 1) return PSTD_OK;
    for (int axis = 0; axis < 3; ++axis) {
        const bool seg = s->prob.sub_core[axis] > 0;
        int ids[16];
        float ms[16];
        const int nv = std::min(16, pass_variants(local_len(s->prob, axis), seg, ids, 16));
        if (nv <= 1) continue;
        pstd_status st = time_shapes(s, axis, ids, nv, reps, ms);
        if (st) return st;
        int best = 0;
        for (int k = 1; k < nv; ++k)
            if (ms[k] < 0.97f * ms[best]) best = k;  // a later shape must win clearly: stable choices
        s->variant[axis] = ids[best];
    }
    solver_drop_graph(s);
    return PSTD_OK;
}

}  // namespace pstd

using namespace pstd;

extern "C" {

pstd_status pstd_problem_init_defaults(pstd_problem* p) {
    if (!p) return PSTD_EINVAL;
    std::memset(p, 0, sizeof(*p));
    const double h = 0.1, k0 = kPi / (4 * h);
    for (int a = 0; a < 3; ++a) {
        p->n[a] = 48;
        p->h[a] = h;
        p->abc_cells[a] = 8;
        p->tfsf[a][0] = 12;
        p->tfsf[a][1] = 18;
        p->tfsf[a][2] = 30;
        p->tfsf[a][3] = 36;
        p->surf_lo[a] = 10;
        p->surf_hi[a] = 38;
    }
    p->hbar = 1.0;
    p->mass = 1.0;
    p->k0 = k0;
    p->abc_U0 = 10.0;
    p->abc_alpha = 0.5;
    p->v_max = 0.5 * k0 * k0 / 2;
    p->ramp_periods = 4.0;
    return PSTD_OK;
}

pstd_status pstd_critical_dt(const pstd_problem* p, double vmax, double* dt_out) {
    if (!p || !dt_out || !(p->hbar > 0 && p->mass > 0) || !(vmax >= 0)) return PSTD_EINVAL;
    double lam = 0;
    for (int a = 0; a < 3; ++a) {
        if (!(p->h[a] > 0)) return PSTD_EINVAL;
        lam += 1.0 / (p->h[a] * p->h[a]);
    }
    lam *= p->hbar * p->hbar * kPi * kPi / (2.0 * p->mass);
    *dt_out = p->hbar / (lam + vmax);
    return PSTD_OK;
}

pstd_status pstd_reduced_step(const pstd_problem* p, double* dtau_out, double* eta_out) {
    if (!p || !dtau_out || !eta_out) return PSTD_EINVAL;
    pstd_status st = validate(p);
    if (st) return st;
    double E0, dxb[3], dtau, eta, crit;
    reduced(p, &E0, dxb, &dtau, &eta, &crit);
    *dtau_out = dtau;
    *eta_out = eta;
    return PSTD_OK;
}

pstd_status pstd_create(const pstd_problem* p, void* hip_stream, pstd_solver** out) {
    if (!out) return PSTD_EINVAL;
    return solver_create(p, (hipStream_t)hip_stream, nullptr, out);
}

pstd_status pstd_set_potential(pstd_solver* s, const float* V_dev, int64_t n_cells) {
    if (!s || !V_dev) return PSTD_EINVAL;
    if (n_cells != s->cells) return fail(s, PSTD_EINVAL, "n_cells does not match the grid");
    adjoint_invalidate(s);
    std::vector<float> V(n_cells);
    HIP_TRY(s, hipMemcpyAsync(V.data(), V_dev, n_cells * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const pstd_problem& p = s->prob;
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    double vmax = 0;
    for (int k = 0; k < nz; ++k) {
        const bool ck = k >= p.tfsf[2][1] && k <= p.tfsf[2][2];
        for (int j = 0; j < ny; ++j) {
            const bool cj = j >= p.tfsf[1][1] && j <= p.tfsf[1][2];
            for (int i = 0; i < nx; ++i) {
                const int64_t id = i + (int64_t)nx * (j + (int64_t)ny * k);
                const double v = V[id];
                if (!std::isfinite(v)) return fail(s, PSTD_ENONFINITE, "non-finite potential value");
                const bool ci = i >= p.tfsf[0][1] && i <= p.tfsf[0][2];
                if (v != 0.0 && !(ci && cj && ck))
                    return fail(s, PSTD_EINVAL, "potential must vanish where the taper is below one");
                vmax = std::max(vmax, std::fabs(v));
            }
        }
    }
    if (vmax > p.v_max * (1 + 1e-6) && !p.force_dt)
        return fail(s, PSTD_EUNSTABLE, "max |V| exceeds v_max used to size the step");
    const std::vector<float> box = scaled_potential(s, V.data());
    HIP_TRY(s, hipMemcpy(s->vbox, box.data(), box.size() * sizeof(float), hipMemcpyHostToDevice));
    if (s->v2full) {
        const std::vector<float> full = scaled_potential_full(s, V.data());
        HIP_TRY(s, hipMemcpy(s->v2full, full.data(), full.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    return PSTD_OK;
}

pstd_status pstd_set_state(pstd_solver* s, const void* prev, const void* cur, int64_t n_cells, int64_t step) {
    if (!s || !prev || !cur || step < 0) return PSTD_EINVAL;
    if (n_cells != s->cells) return fail(s, PSTD_EINVAL, "n_cells does not match the grid");
    adjoint_invalidate(s);
    pstd_status st = solver_ensure_tables(s, step + 1);
    if (st) return st;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    HIP_TRY(s, hipMemcpy(s->buf[(step + 1) & 1], prev, n_cells * sizeof(float2), hipMemcpyDeviceToDevice));
    HIP_TRY(s, hipMemcpy(s->buf[step & 1], cur, n_cells * sizeof(float2), hipMemcpyDeviceToDevice));
    for (int a = 0; a < 3; ++a) HIP_TRY(s, hipMemset(s->acc[a], 0, 8 * s->points[a] * sizeof(double2)));
    HIP_TRY(s, sphere_clear(s, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const int64_t c[2] = {step, std::numeric_limits<int64_t>::max()};
    HIP_TRY(s, hipMemcpy(s->ctr, c, sizeof(c), hipMemcpyHostToDevice));
    HIP_TRY(s, hipDeviceSynchronize());
    s->step = step;
    s->inc_sum = 0;
    s->win_steps = 0;
    pulse_reset(s);
    return PSTD_OK;
}

pstd_status pstd_run(pstd_solver* s, int64_t n_steps) {
    if (!s || n_steps < 0) return PSTD_EINVAL;
    if (s->in_batch) return fail(s, PSTD_ESTATE, "instances of a batch are stepped by the batch");
    adjoint_invalidate(s);
    pstd_status st = solver_ensure_tables(s, s->step + n_steps);
    if (st) return st;
    int64_t left = n_steps;
    if (left >= kGraphSteps) {
        if ((st = build_graph(s))) return st;
        for (; left >= kGraphSteps; left -= kGraphSteps) HIP_TRY(s, hipGraphLaunch(s->graph, s->stream));
    }
    if (left > 0 && (st = launch_steps(s, s->stream, (int)left, nullptr))) return st;
    solver_account_steps(s, s->step, s->step + n_steps);
    s->step += n_steps;
    return PSTD_OK;
}

pstd_status pstd_run_timed(pstd_solver* s, int64_t n_steps, double* pass_ms) {
    if (!s || n_steps < 0 || !pass_ms) return PSTD_EINVAL;
    if (s->in_batch) return fail(s, PSTD_ESTATE, "instances of a batch are stepped by the batch");
    adjoint_invalidate(s);
    pstd_status st = solver_ensure_tables(s, s->step + n_steps);
    if (st) return st;
    // one pair of events around every pass launch, all steps queued back to
    // back (as pstd_run does), read after the last one
    std::vector<hipEvent_t> ev(6 * (size_t)n_steps, nullptr);
    auto destroy = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto& e : ev)
        if (hipError_t r = hipEventCreate(&e)) {
            destroy();
            return hip_fail(s, r, "hipEventCreate");
        }
    double sum[3] = {0, 0, 0};
    int64_t done = 0;
    for (; done < n_steps; ++done) {
        st = launch_steps(s, s->stream, 1, &ev[6 * (size_t)done]);
        if (st) break;
    }
    if (!st && done > 0) {
        hipError_t e = hipEventSynchronize(ev[6 * (size_t)(done - 1) + 5]);
        if (e) st = hip_fail(s, e, "event sync");
    }
    for (int64_t k = 0; k < done && !st; ++k)
        for (int a = 0; a < 3; ++a) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev[6 * (size_t)k + 2 * a], ev[6 * (size_t)k + 2 * a + 1]);
            sum[a] += ms;
        }
    destroy();
    solver_account_steps(s, s->step, s->step + done);
    s->step += done;
    for (int a = 0; a < 3; ++a) pass_ms[a] = sum[a];
    return st;
}

}  // extern "C"

namespace {

// The FP64 norms of psi^n and psi^{n-1} through `d` (2 norm_scratch_doubles()
// doubles of device memory); synchronises the solver's stream.
pstd_status check_state_with(pstd_solver* s, double* d, double* norm2_out) {
    const int m = norm_scratch_doubles();
    double h[2] = {0, 0};
    hipError_t e = launch_norm(s->buf[s->step & 1], s->cells, d, s->stream);          // psi^n
    if (!e) e = launch_norm(s->buf[(s->step + 1) & 1], s->cells, d + m, s->stream);   // psi^{n-1}
    if (!e) e = hipMemcpyAsync(&h[0], d, sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (!e) e = hipMemcpyAsync(&h[1], d + m, sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (!e) e = hipStreamSynchronize(s->stream);
    if (e) return hip_fail(s, e, "state check");
    *norm2_out = h[0];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]))
        return fail(s, PSTD_ENONFINITE, "the wave function holds NaN or Inf values");
    return PSTD_OK;
}

}  // namespace

extern "C" {

pstd_status pstd_check_state(pstd_solver* s, double* norm2_out) {
    if (!s || !norm2_out) return PSTD_EINVAL;
    double* d = nullptr;
    HIP_TRY(s, hipMalloc(&d, 2 * norm_scratch_doubles() * sizeof(double)));
    const pstd_status st = check_state_with(s, d, norm2_out);
    (void)hipFree(d);
    return st;
}

pstd_status pstd_check_state_noalloc(pstd_solver* s, double* norm2_out) {
    if (!s || !norm2_out) return PSTD_EINVAL;
    const int need = 2 * norm_scratch_doubles();
    if (need > kStaticScratchDoubles)
        return fail(s, PSTD_EINVAL, "state check: the reduction needs " + std::to_string(need) +
                                        " doubles of scratch, more than the static " +
                                        std::to_string(kStaticScratchDoubles));
    if (s->device < 0 || s->device >= kMaxDevices) return fail(s, PSTD_EINVAL, "state check: device out of range");
    // one call at a time in this process uses a device's array
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    double* d = g_scratch_dev[s->device];
    if (!d) return fail(s, PSTD_ESTATE, "state check: no static scratch address for this device");
    return check_state_with(s, d, norm2_out);
}

pstd_status pstd_pass_time(pstd_solver* s, int32_t axis, int32_t reps, double* us_out) {
    if (!s || !us_out || axis < 0 || axis > 2 || reps < 1) return PSTD_EINVAL;
    float ms = 0;
    pstd_status st = time_shapes(s, axis, &s->variant[axis], 1, reps, &ms);
    if (st) return st;
    *us_out = 1e3 * ms;
    return PSTD_OK;
}

pstd_status pstd_autotune(pstd_solver* s, int32_t reps) {
    if (!s || reps < 1) return PSTD_EINVAL;
    pstd_status st = solver_autotune(s, reps);
    // capture the step graph of the chosen shapes now, not in the next run
    if (!st && !s->in_batch) st = build_graph(s);
    return st;
}

pstd_status pstd_tile_info(const pstd_solver* s, int32_t axis, int32_t* info_host) {
    if (!s || !info_host || axis < 0 || axis > 2) return PSTD_EINVAL;
    const PassShape sh = variant_shape(s->variant[axis]);
    info_host[0] = sh.N;
    info_host[1] = sh.N1;
    info_host[2] = sh.N2;
    info_host[3] = sh.P;
    info_host[4] = sh.M1;
    return PSTD_OK;
}

pstd_status pstd_set_tile(pstd_solver* s, int32_t axis, int32_t n1, int32_t pencils, int32_t m1) {
    if (!s || axis < 0 || axis > 2) return PSTD_EINVAL;
    const bool seg = s->prob.sub_core[axis] > 0;
    int ids[16];
    const int nv = std::min(16, pass_variants(local_len(s->prob, axis), seg, ids, 16));
    for (int k = 0; k < nv; ++k) {
        const PassShape sh = variant_shape(ids[k]);
        if (sh.N1 == n1 && sh.P == pencils && sh.M1 == m1) {
            HIP_TRY(s, hipStreamSynchronize(s->stream));
            s->variant[axis] = ids[k];
            solver_drop_graph(s);
            return PSTD_OK;
        }
    }
    return fail(s, PSTD_EUNSUPPORTED, "no compiled tile shape with that factor, pencil count and stage-B split");
}

pstd_status pstd_tile_variants(int32_t n, int32_t segmented, int32_t* shapes_host, int32_t cap, int32_t* count_out) {
    if (!count_out || cap < 0 || (cap > 0 && !shapes_host)) return PSTD_EINVAL;
    int ids[16];
    const int nv = std::min(16, pass_variants(n, segmented != 0, ids, 16));
    for (int k = 0; k < nv && k < cap; ++k) {
        const PassShape sh = variant_shape(ids[k]);
        shapes_host[4 * k] = sh.N1;
        shapes_host[4 * k + 1] = sh.N2;
        shapes_host[4 * k + 2] = sh.P;
        shapes_host[4 * k + 3] = sh.M1;
    }
    *count_out = nv;
    return PSTD_OK;
}

pstd_status pstd_step_index(const pstd_solver* s, int64_t* out) {
    if (!s || !out) return PSTD_EINVAL;
    *out = s->step;
    return PSTD_OK;
}

pstd_status pstd_get_psi(pstd_solver* s, int32_t level, void* psi_dev, int64_t n_cells) {
    if (!s || !psi_dev || (level != 0 && level != 1)) return PSTD_EINVAL;
    if (n_cells != s->cells) return fail(s, PSTD_EINVAL, "n_cells does not match the grid");
    const float2* src = s->buf[(s->step + (level == 0 ? 0 : 1)) & 1];
    HIP_TRY(s, hipMemcpyAsync(psi_dev, src, n_cells * sizeof(float2), hipMemcpyDeviceToDevice, s->stream));
    return PSTD_OK;
}

// serialized state: header, psi^{n-1}, psi^n, the surface DFT sums (value
// and compensation) of the three axes, the sphere's sums (one set per
// wavenumber), a pulsed run's per-wavenumber box sums
struct StateHeader {
    int64_t magic;
    int64_t n[3];
    int64_t step;
    double inc_sum;
    int64_t bytes;
    int64_t n_k;     // wavenumbers of a pulsed run, 0 without a pulse
    int64_t from;    // pulsed run: first step since the pulse was set or pstd_set_state
    int64_t pad;
};
constexpr int64_t kStateMagic = 0x3276534454535050LL;  // "PPSTDSv2"

static int64_t state_bytes(const pstd_solver* s) {
    int64_t b = (int64_t)sizeof(StateHeader) + 2 * s->cells * (int64_t)sizeof(float2);
    for (int a = 0; a < 3; ++a) b += 8 * s->points[a] * (int64_t)sizeof(double2);
    return b + sphere_state_bytes(s) + pulse_state_bytes(s);
}

pstd_status pstd_state_size(const pstd_solver* s, int64_t* bytes_out) {
    if (!s || !bytes_out) return PSTD_EINVAL;
    *bytes_out = state_bytes(s);
    return PSTD_OK;
}

pstd_status pstd_save_state(pstd_solver* s, void* dev_buf, int64_t bytes) {
    if (!s || !dev_buf) return PSTD_EINVAL;
    const int64_t need = state_bytes(s);
    if (bytes < need) return fail(s, PSTD_EINVAL, "buffer smaller than pstd_state_size");
    const int64_t n_k = (s->pulse ? pulse_wavenumbers(s) : 0);
    StateHeader h{kStateMagic, {s->prob.n[0], s->prob.n[1], s->prob.n[2]}, s->step, s->inc_sum, need, n_k,
                  n_k ? pulse_from(s) : 0, 0};
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    char* d = (char*)dev_buf;
    HIP_TRY(s, hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice));
    d += sizeof(h);
    const size_t fb = s->cells * sizeof(float2);
    HIP_TRY(s, hipMemcpyAsync(d, s->buf[(s->step + 1) & 1], fb, hipMemcpyDeviceToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(d + fb, s->buf[s->step & 1], fb, hipMemcpyDeviceToDevice, s->stream));
    d += 2 * fb;
    for (int a = 0; a < 3; ++a) {
        const size_t ab = 8 * s->points[a] * sizeof(double2);
        HIP_TRY(s, hipMemcpyAsync(d, s->acc[a], ab, hipMemcpyDeviceToDevice, s->stream));
        d += ab;
    }
    HIP_TRY(s, sphere_save(s, d, s->stream));
    HIP_TRY(s, pulse_save(s, d + sphere_state_bytes(s), s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return PSTD_OK;
}

pstd_status pstd_load_state(pstd_solver* s, const void* dev_buf, int64_t bytes) {
    if (!s || !dev_buf) return PSTD_EINVAL;
    if (s->in_batch) return fail(s, PSTD_ESTATE, "instances of a batch are stepped by the batch");
    const int64_t need = state_bytes(s);
    if (bytes < need) return fail(s, PSTD_EINVAL, "buffer smaller than pstd_state_size");
    StateHeader h{};
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    HIP_TRY(s, hipMemcpy(&h, dev_buf, sizeof(h), hipMemcpyDeviceToHost));
    if (h.magic != kStateMagic || h.bytes != need || h.n[0] != s->prob.n[0] || h.n[1] != s->prob.n[1] ||
        h.n[2] != s->prob.n[2] || h.step < 0 || !(h.inc_sum >= 0))
        return fail(s, PSTD_EINVAL, "buffer does not hold a saved state of this grid");
    if (h.n_k != (s->pulse ? pulse_wavenumbers(s) : 0) || (h.n_k && (h.from < 0 || h.from > h.step)))
        return fail(s, PSTD_EINVAL, "the saved run and this solver differ in their pulse");
    adjoint_invalidate(s);
    pstd_status st = solver_ensure_tables(s, h.step + 1);
    if (st) return st;
    const char* d = (const char*)dev_buf + sizeof(h);
    const size_t fb = s->cells * sizeof(float2);
    HIP_TRY(s, hipMemcpyAsync(s->buf[(h.step + 1) & 1], d, fb, hipMemcpyDeviceToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->buf[h.step & 1], d + fb, fb, hipMemcpyDeviceToDevice, s->stream));
    d += 2 * fb;
    for (int a = 0; a < 3; ++a) {
        const size_t ab = 8 * s->points[a] * sizeof(double2);
        HIP_TRY(s, hipMemcpyAsync(s->acc[a], d, ab, hipMemcpyDeviceToDevice, s->stream));
        d += ab;
    }
    HIP_TRY(s, sphere_load(s, d, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const int64_t c[2] = {h.step, std::numeric_limits<int64_t>::max()};
    HIP_TRY(s, hipMemcpy(s->ctr, c, sizeof(c), hipMemcpyHostToDevice));
    s->step = h.step;
    s->inc_sum = h.inc_sum;
    s->win_steps = h.inc_sum > 0 ? 1 : 0;
    if (h.n_k) {
        // the window steps since the pulse's first step, and its table of this step
        s->win_steps = std::max<int64_t>(0, std::min(h.step, s->prob.dft_end) - std::max(h.from, s->prob.dft_begin));
        HIP_TRY(s, pulse_load(s, d + sphere_state_bytes(s), h.from));
    }
    return PSTD_OK;
}

pstd_status pstd_surface_size(const pstd_solver* s, int64_t* n_out) {
    if (!s || !n_out) return PSTD_EINVAL;
    *n_out = 4 * (s->points[0] + s->points[1] + s->points[2]);
    return PSTD_OK;
}

pstd_status pstd_get_surface_phasors_k(pstd_solver* s, int32_t ik, double* out_dev, int64_t n) {
    if (!s || !out_dev) return PSTD_EINVAL;
    int64_t need;
    pstd_surface_size(s, &need);
    if (n != need) return fail(s, PSTD_EINVAL, "output size must equal pstd_surface_size");
    if (s->sphere) return fail(s, PSTD_ESTATE, "the problem integrates over the sphere (pstd_get_sphere_phasors)");
    if (!(s->pulse ? s->win_steps > 0 : s->inc_sum > 0)) return fail(s, PSTD_ESTATE, "no step of the DFT window has run");
    hipError_t e;
    if (s->pulse) {
        BoxOut o;
        if (pstd_status st = pulse_box_output(s, ik, false, &o)) return st;
        e = finalize_phasors(o.acc, s->points, o.scale, (double2*)out_dev, s->stream);
    } else {
        if (ik != 0) return fail(s, PSTD_EINVAL, "without a pulse the only wavenumber index is 0");
        e = finalize_phasors(s->acc, s->points, real_scale(1.0 / s->inc_sum), (double2*)out_dev, s->stream);
    }
    if (e) return hip_fail(s, e, "finalize_phasors");
    return PSTD_OK;
}

pstd_status pstd_get_surface_phasors(pstd_solver* s, double* out_dev, int64_t n) {
    return pstd_get_surface_phasors_k(s, 0, out_dev, n);
}

pstd_status pstd_sphere_size(const pstd_solver* s, int64_t* n_nodes_out) {
    if (!s || !n_nodes_out) return PSTD_EINVAL;
    *n_nodes_out = sphere_nodes(s);
    return PSTD_OK;
}

namespace {

// a window step has run (with a pulse the ramp plays no part)
bool window_ran(const pstd_solver* s) { return s->pulse ? s->win_steps > 0 : s->inc_sum > 0; }

}  // namespace

pstd_status pstd_get_sphere_phasors_k(pstd_solver* s, int32_t ik, double* out_dev, int64_t n) {
    if (!s || !out_dev) return PSTD_EINVAL;
    if (!s->sphere) return fail(s, PSTD_ESTATE, "the problem has no spherical surface");
    if (n != 2 * sphere_nodes(s)) return fail(s, PSTD_EINVAL, "output size must be twice pstd_sphere_size");
    if (!window_ran(s)) return fail(s, PSTD_ESTATE, "no step of the DFT window has run");
    SphereOut o;
    if (pstd_status st = pulse_output(s, ik, &o)) return st;
    hipError_t e = sphere_phasors(s, o, (double2*)out_dev, s->stream);
    if (e) return hip_fail(s, e, "sphere phasors");
    return PSTD_OK;
}

pstd_status pstd_get_sphere_phasors(pstd_solver* s, double* out_dev, int64_t n) {
    return pstd_get_sphere_phasors_k(s, 0, out_dev, n);
}

pstd_status pstd_project_k(pstd_solver* s, int32_t ik, const double* obs_dev, int64_t n_obs, double* out_dev) {
    if (!s || n_obs < 0 || (n_obs > 0 && (!obs_dev || !out_dev))) return PSTD_EINVAL;
    if (n_obs == 0) return PSTD_OK;  // nothing to evaluate
    if (!window_ran(s)) return fail(s, PSTD_ESTATE, "no step of the DFT window has run");
    if (s->sphere) {
        SphereOut o;
        if (pstd_status st = pulse_output(s, ik, &o)) return st;
        // the Kirchhoff integral holds outside the sphere only
        std::vector<double> h(3 * n_obs);
        HIP_TRY(s, hipMemcpyAsync(h.data(), obs_dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        for (int64_t o = 0; o < n_obs; ++o) {
            const double r = std::sqrt(h[3 * o] * h[3 * o] + h[3 * o + 1] * h[3 * o + 1] + h[3 * o + 2] * h[3 * o + 2]);
            if (!(r > s->prob.sphere_radius)) return fail(s, PSTD_EINVAL, "observation point inside the sphere or not finite");
        }
        hipError_t e = sphere_project(s, o, (const double3*)obs_dev, n_obs, (double2*)out_dev, s->stream);
        if (e) return hip_fail(s, e, "sphere projection");
        return PSTD_OK;
    }
    std::string msg;
    if (s->pulse) {
        BoxOut o;
        if (pstd_status st = pulse_box_output(s, ik, true, &o)) return st;
        hipError_t e = project_points(o.proj, o.prob, o.dxb, o.acc, s->points, o.scale, (const double3*)obs_dev, n_obs,
                                      (double2*)out_dev, s->stream, &msg);
        if (e) return msg.empty() ? hip_fail(s, e, "project") : fail(s, PSTD_EINVAL, msg);
        return PSTD_OK;
    }
    if (ik != 0) return fail(s, PSTD_EINVAL, "without a pulse the only wavenumber index is 0");
    hipError_t e = project_points(&s->proj, s->prob, s->dxb, s->acc, s->points, real_scale(1.0 / s->inc_sum),
                                  (const double3*)obs_dev, n_obs, (double2*)out_dev, s->stream, &msg);
    if (e) return msg.empty() ? hip_fail(s, e, "project") : fail(s, PSTD_EINVAL, msg);
    return PSTD_OK;
}

pstd_status pstd_project(pstd_solver* s, const double* obs_dev, int64_t n_obs, double* out_dev) {
    return pstd_project_k(s, 0, obs_dev, n_obs, out_dev);
}

pstd_status pstd_far_field_k(pstd_solver* s, int32_t ik, const double* dir_dev, int64_t n_dir, double* out_dev) {
    if (!s || n_dir < 0 || (n_dir > 0 && (!dir_dev || !out_dev))) return PSTD_EINVAL;
    if (n_dir == 0) return PSTD_OK;  // nothing to evaluate
    if (!window_ran(s)) return fail(s, PSTD_ESTATE, "no step of the DFT window has run");
    if (s->sphere) {
        SphereOut o;
        if (pstd_status st = pulse_output(s, ik, &o)) return st;
        hipError_t e = sphere_far_field(s, o, (const double3*)dir_dev, n_dir, (double2*)out_dev, s->stream);
        if (e) return hip_fail(s, e, "sphere far field");
        return PSTD_OK;
    }
    std::string msg;
    if (s->pulse) {
        BoxOut o;
        if (pstd_status st = pulse_box_output(s, ik, true, &o)) return st;
        hipError_t e = far_field(o.proj, o.prob, o.dxb, o.acc, s->points, o.scale, (const double3*)dir_dev, n_dir,
                                 (double2*)out_dev, s->stream, &msg);
        if (e) return msg.empty() ? hip_fail(s, e, "far_field") : fail(s, PSTD_EINVAL, msg);
        return PSTD_OK;
    }
    if (ik != 0) return fail(s, PSTD_EINVAL, "without a pulse the only wavenumber index is 0");
    hipError_t e = far_field(&s->proj, s->prob, s->dxb, s->acc, s->points, real_scale(1.0 / s->inc_sum),
                             (const double3*)dir_dev, n_dir, (double2*)out_dev, s->stream, &msg);
    if (e) return msg.empty() ? hip_fail(s, e, "far_field") : fail(s, PSTD_EINVAL, msg);
    return PSTD_OK;
}

pstd_status pstd_far_field(pstd_solver* s, const double* dir_dev, int64_t n_dir, double* out_dev) {
    return pstd_far_field_k(s, 0, dir_dev, n_dir, out_dev);
}

pstd_status pstd_set_pulse(pstd_solver* s, const double* psi0_host, int32_t n1d, double delta, const double* kbar_host,
                           int32_t n_k) {
    if (!s) return PSTD_EINVAL;
    adjoint_invalidate(s);
    solver_drop_graph(s);
    return pulse_set(s, psi0_host, n1d, delta, kbar_host, n_k);
}

pstd_status pstd_destroy(pstd_solver* s) {
    if (!s) return PSTD_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    solver_drop_graph(s);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    (void)hipFree(s->buf[0]);
    (void)hipFree(s->buf[1]);
    (void)hipFree(s->L);
    (void)hipFree(s->vbox);
    (void)hipFree(s->v2full);
    (void)hipFree(s->wr);
    (void)hipFree(s->tables);
    (void)hipFree(s->sigma_tab);
    (void)hipFree(s->w_tab);
    (void)hipFree(s->dft_tab);
    (void)hipFree(s->dft_zero);
    if (s->owns_ctr) (void)hipFree(s->ctr);
    for (int a = 0; a < 3; ++a) (void)hipFree(s->acc[a]);
    project_free(s->proj);
    adjoint_free(s);
    sphere_free(s->sphere);
    pulse_free(s->pulse);
    delete s;
    return PSTD_OK;
}

const char* pstd_status_string(pstd_status st) {
    switch (st) {
        case PSTD_OK: return "PSTD_OK";
        case PSTD_EINVAL: return "PSTD_EINVAL";
        case PSTD_EUNSTABLE: return "PSTD_EUNSTABLE";
        case PSTD_ENONFINITE: return "PSTD_ENONFINITE";
        case PSTD_ENOMEM: return "PSTD_ENOMEM";
        case PSTD_EHIP: return "PSTD_EHIP";
        case PSTD_ESTATE: return "PSTD_ESTATE";
        case PSTD_EUNSUPPORTED: return "PSTD_EUNSUPPORTED";
    }
    return "PSTD_UNKNOWN";
}

const char* pstd_last_error(const pstd_solver* s) {
    return s ? s->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
