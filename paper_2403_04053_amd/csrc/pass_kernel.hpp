// Pencil passes of the PSTD step (Eq. PSTDupdating, Section 2.5).
//
// A pass along axis a computes F_a^-1[kbar_a^2 F_a psi^n] for every pencil
// along a.  Each pencil of length N = N1 N2 is handled by N2 threads in stage
// A (N1-point DFTs over stride-N2 elements, held in VGPRs) and by N1 threads
// in stage B (N2-point DFTs), with one padded LDS exchange between the two
// stages and one back.  The forward transform leaves the spectrum in stage-B
// order k1 + N1 k2, where it is scaled by the kbar^2 table; the inverse runs
// the same stages backwards, so no digit-reversal pass is needed and the
// result returns to the registers it was loaded into.
//
// Where N1 < N2, N2 - N1 of a pencil's threads idle in stage B.  Shapes with
// M1 > 0 split stage B once more, N2 = M1 M2 (M1 and M2 both dividing N1):
// every thread of the pencil does N1/M1 M1-point DFTs (B1), then, after a
// second exchange in the same LDS rows, N1/M2 M2-point DFTs (B2) with the
// kbar^2 scaling between the forward and inverse M2-point DFTs; so all N2
// threads work in every stage and no thread holds more than N1 elements.
//
// Loads and stores are coalesced without an LDS transpose: the x pass gives
// consecutive lanes consecutive elements of a row; the y and z passes give
// consecutive lanes consecutive x of a tile of P pencils.  The per-axis
// twiddles and kbar^2 are staged in LDS once per workgroup, and so are the
// derivative rows of the surface planes (used only inside the DFT window)
// for N <= 200; longer pencils read those rows from global memory, where
// neighbouring lanes read neighbouring entries, to keep their occupancy.
//
// Epilogues: x pass writes L; y pass adds to L (which it reads at the start,
// with the field); z pass adds its term and applies the leapfrog update with
// the potential (V read only on the pencils that cross the box where it may
// be non-zero), TF/SF source and absorber, writing psi^{n+1} over psi^{n-1}.
// When that box covers few rows (PassArgs::potx), the x pass takes the
// potential term instead, on the rows that cross the box, and the z pass
// holds no copy of psi^n through its transforms.
// Inside the DFT window each pass also accumulates, in FP64 with Neumaier
// compensation, the DFT of psi and of its spectral normal derivative on the
// two planes normal to its axis (Eqs. psiphasor, dpsiphasor).
//
// Order and caches: workgroups are mapped to tiles so that each of the 8
// XCDs walks a contiguous run of tiles; the x and y passes both number their
// tiles plane by plane, so an XCD meets the same planes in both, and the y
// pass walks its run backwards, starting on the lines its x pass wrote last.
// For fields beyond the Infinity Cache the z pass reads its last-use
// operands with non-temporal loads (NTL), leaving the cache to the
// psi^{n+1} it writes for the next step's x pass.
//
// Segmented mode (overlapping subdomains, Section 2.6): a pencil is split
// into segments of C core points; each segment is transformed as a local
// array of N = C + 2H points read from the global array with the halo
// weights, and only its core points are written.
//
// This header holds the kernel and its launch templates; pass_variants.hpp
// lists the compiled tile shapes, each instantiated in one of the
// pass_inst<k>.hip units (so that the shapes compile in parallel), and
// pass.hip holds the table the host code picks them from.
#pragma once

#include <algorithm>

#include "dft.hpp"
#include "internal.hpp"

namespace pstd {

__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

// Pointers into device global memory.  The descriptor may come from the
// kernel arguments or from a table in memory; qualifying every pointer keeps
// the loads and stores global (not flat) either way.
#if defined(__HIP_DEVICE_COMPILE__)
#define GMEM __attribute__((address_space(1)))
#else
#define GMEM
#endif
template <class T>
__device__ __forceinline__ GMEM T* gmem(T* p) { return (GMEM T*)p; }

// a value's last use in this step, read with a non-temporal load when NTL:
// fields beyond the Infinity Cache then leave it to the lines the next pass
// reads (within the cache the hint costs time, so it is a launch choice: NTL)
typedef float float2_vec __attribute__((ext_vector_type(2)));
template <bool NTL>
__device__ __forceinline__ float2 load_last(GMEM const float2* p) {
    if constexpr (NTL) {
        const float2_vec v = __builtin_nontemporal_load((GMEM const float2_vec*)p);
        return make_float2(v.x, v.y);
    } else {
        return *p;
    }
}

using PtrF2 = float2*;
using CPtrF2 = const float2*;

// the descriptor fields a pass uses, copied once into (uniform) registers
struct Fields {
    GMEM const int64_t* ctr;
    GMEM float2* buf0;
    GMEM float2* buf1;
    GMEM float2* L;
    GMEM const float* vbox;
    int vlo0, vlo1, vlo2, vn0, vn1, vn2;
    GMEM const float *wr0, *wr1, *wr2;
    int nx, ny, nz;
    GMEM const float *kk, *gam;
    GMEM const float2 *tw, *zt, *dz, *dlo, *dhi;
    GMEM const float4* zd;
    GMEM const float2 *zt_x, *dz_x, *zt_y, *dz_y;
    GMEM const float *gam_x, *gam_y;
    GMEM const float2* sigma_tab;
    GMEM const double2* w_tab;
    GMEM const int* dft_tab;
    int plane_lo, plane_hi, seg_plane0, seg_plane1;
    GMEM double2* acc;
    GMEM float2* bstage;
    int64_t points;
    int seg_core, seg_halo, nseg;
    GMEM const float* wloc;
    int ntx;
    GMEM const float2 *inj_lo_p, *inj_lo_d, *inj_hi_p, *inj_hi_d;
    GMEM const CPtrF2* fwd_tab;
    GMEM float* grad;
    GMEM const PtrF2* stash_tab;
};

template <int AXIS>
__device__ __forceinline__ Fields fields(const PassArgs& a) {
    Fields f;
    f.ctr = gmem(a.ctr);
    f.buf0 = gmem(a.buf[0]);
    f.buf1 = gmem(a.buf[1]);
    f.L = gmem(a.L);
    f.vbox = gmem(a.pot.box);
    f.vlo0 = a.pot.lo[0];
    f.vlo1 = a.pot.lo[1];
    f.vlo2 = a.pot.lo[2];
    f.vn0 = a.pot.n[0];
    f.vn1 = a.pot.n[1];
    f.vn2 = a.pot.n[2];
    f.wr0 = gmem(a.pot.wr[0]);
    f.wr1 = gmem(a.pot.wr[1]);
    f.wr2 = gmem(a.pot.wr[2]);
    f.nx = a.nx;
    f.ny = a.ny;
    f.nz = a.nz;
    f.kk = gmem(a.ax[AXIS].kk);
    f.gam = gmem(a.ax[AXIS].gam);
    f.tw = gmem(a.ax[AXIS].tw);
    f.zt = gmem(a.ax[AXIS].zt);
    f.dz = gmem(a.ax[AXIS].dz);
    f.zd = gmem(a.ax[AXIS].zd);
    f.dlo = gmem(a.ax[AXIS].dlo);
    f.dhi = gmem(a.ax[AXIS].dhi);
    f.zt_x = gmem(a.ax[0].zt);
    f.dz_x = gmem(a.ax[0].dz);
    f.zt_y = gmem(a.ax[1].zt);
    f.dz_y = gmem(a.ax[1].dz);
    f.gam_x = gmem(a.ax[0].gam);
    f.gam_y = gmem(a.ax[1].gam);
    f.sigma_tab = gmem(a.sigma_tab);
    f.w_tab = gmem(a.w_tab);
    f.dft_tab = gmem(a.dft_tab);
    f.plane_lo = a.plane_lo;
    f.plane_hi = a.plane_hi;
    f.seg_plane0 = a.seg_plane[0];
    f.seg_plane1 = a.seg_plane[1];
    f.acc = gmem(a.acc);
    f.bstage = gmem(a.bstage);
    f.points = a.points;
    f.seg_core = a.seg_core;
    f.seg_halo = a.seg_halo;
    f.nseg = a.nseg;
    f.wloc = gmem(a.wloc);
    f.ntx = a.ntx;
    f.inj_lo_p = gmem(a.inj_lo_p);
    f.inj_lo_d = gmem(a.inj_lo_d);
    f.inj_hi_p = gmem(a.inj_hi_p);
    f.inj_hi_d = gmem(a.inj_hi_d);
    f.fwd_tab = gmem(a.fwd_tab);
    f.grad = gmem(a.grad);
    f.stash_tab = gmem(a.stash_tab);
    return f;
}

// Pencil geometry of one tile: element e of pencil pA lives at
// base + e * estride (segmented pencils: e is a local index, global index g0 + e)
struct TileGeo {
    int64_t base, estride;
    bool valid;
    int seg, g0, Ng;
    int px, py;   // (x, y) of the pencil (z pass update)
    int tx, tq;   // x tile and (other, segment) of the y, z passes
};

template <int N, int P, int AXIS, bool SEG>
__device__ __forceinline__ TileGeo tile_geo(const Fields& f, int tile, int pA, bool activeA) {
    TileGeo g;
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    const int C = SEG ? f.seg_core : N;
    const int H = SEG ? f.seg_halo : 0;
    const int nseg = SEG ? f.nseg : 1;
    g.px = 0;
    g.py = 0;
    g.tx = 0;
    g.tq = 0;
    if constexpr (AXIS == 0) {
        const int64_t q = (int64_t)tile * P + pA;
        const int64_t row = q / nseg;
        g.seg = (int)(q % nseg);
        g.valid = activeA && q < (int64_t)ny * nz * nseg;
        g.base = row * nx + (g.seg * C - H);
        g.estride = 1;
        g.Ng = nx;
    } else if constexpr (AXIS == 1) {
        g.tx = tile % f.ntx;
        g.tq = tile / f.ntx;
        const int x = g.tx * P + pA;
        const int z = g.tq / nseg;
        g.seg = g.tq % nseg;
        g.valid = activeA && x < nx;
        g.estride = nx;
        g.base = x + (int64_t)nx * ny * z + (int64_t)(g.seg * C - H) * g.estride;
        g.Ng = ny;
    } else {
        g.tx = tile % f.ntx;
        g.tq = tile / f.ntx;
        g.px = g.tx * P + pA;
        g.py = g.tq / nseg;
        g.seg = g.tq % nseg;
        g.valid = activeA && g.px < nx;
        g.estride = (int64_t)nx * ny;
        g.base = g.px + (int64_t)nx * g.py + (int64_t)(g.seg * C - H) * g.estride;
        g.Ng = nz;
    }
    g.g0 = g.seg * C - H;
    return g;
}

// raw pencil values of one tile (zero outside the grid and for idle lanes)
template <int N, int N1, int N2, bool SEG, bool NTL = false>
__device__ __forceinline__ void load_tile(GMEM const float2* __restrict__ psi, const TileGeo& g, int n2,
                                          float2 (&x)[N1]) {
    unroll<N1>([&](auto i) {
        constexpr int n1 = decltype(i)::value;
        const int e = n2 + N2 * n1;
        const bool in = g.valid && (e < N) && (!SEG || (g.g0 + e >= 0 && g.g0 + e < g.Ng));
        float2 val = make_float2(0.f, 0.f);
        if (in) val = load_last<NTL>(psi + g.base + (int64_t)e * g.estride);
        x[n1] = val;
    });
}

// One workgroup per tile of P pencils; MULTI launches find their instance
// from the prefix table of tiles.
template <int N, int N1, int N2, int M1, int P, int AXIS, bool SEG, bool MULTI, bool ADJ, bool POTX = false,
          bool NTL = false>
__global__ __launch_bounds__(P * (N1 > N2 ? N1 : N2)) void pass_kernel(PassArgs single,
                                                                       const PassArgs* __restrict__ descs,
                                                                       const int* __restrict__ off, int ninst,
                                                                       int koff) {
    constexpr int NT = P * (N1 > N2 ? N1 : N2);
    constexpr int ROW = N2 + 1;                 // padded exchange row
    // odd pencil stride (float2); also holds the four DFT partials per thread
    constexpr int STRIDE = (N1 * ROW > 4 * N2 ? N1 * ROW : 4 * N2) | 1;
    __shared__ float2 ex[P * STRIDE];
    __shared__ float2 s_tw[N];
    __shared__ float s_kk[N];
    // derivative rows of the surface planes: staged in LDS where that costs
    // no occupancy (N <= 200), read from global memory otherwise
    constexpr bool kRowsInLds = N <= 200;
    __shared__ float2 s_dl[kRowsInLds ? N : 1], s_dh[kRowsInLds ? N : 1];

    const int t = threadIdx.x;
    const bool activeA = t < P * N2;
    const int pA = AXIS == 0 ? t / N2 : t % P;
    const int n2 = AXIS == 0 ? t % N2 : t / P;

    // Workgroups are dealt round-robin to the 8 XCDs (blockIdx mod 8); give
    // each XCD a contiguous run of tiles instead, so that neighbouring tiles,
    // which share cache lines (the 4-byte potential of a 16-pencil tile is
    // half a 128-byte line), meet in the same L2.  A bijection of [0, G).
    // The y pass walks each XCD's run backwards: the x pass gave that XCD the
    // same planes and ended on the lines it wrote last, which are still in
    // its L2 and in the Infinity Cache.
    const int G = (int)gridDim.x, gb = (int)blockIdx.x, xcd = gb & 7;
    const int run0 = xcd * (G >> 3) + min(xcd, G & 7), runlen = (G >> 3) + (xcd < (G & 7) ? 1 : 0);
    const int gt = run0 + (AXIS == 1 && !MULTI ? runlen - 1 - (gb >> 3) : (gb >> 3));

    // instance of this workgroup (uniform), its tile, its step: the base
    // counter plus this launch's offset in its group of steps
    Fields f;
    int tile;
    if constexpr (!MULTI) {
        f = fields<AXIS>(single);
        tile = gt;
    } else {
        int inst = 0;
        for (int i = 1; i < ninst; ++i)
            if (gt >= off[i]) inst = i;
        f = fields<AXIS>(descs[inst]);
        tile = gt - off[inst];
    }
    const int64_t nstep = f.ctr[0] + koff;
    if (nstep >= f.ctr[1]) return;  // whole workgroup, before any barrier
    const bool surf = f.dft_tab[nstep] != 0;
    GMEM const float2* __restrict__ psi = (nstep & 1) ? f.buf1 : f.buf0;
    GMEM float2* __restrict__ psi_old = (nstep & 1) ? f.buf0 : f.buf1;

    // tables to LDS (issued before the field loads)
    for (int i = t; i < N; i += NT) {
        s_tw[i] = f.tw[i];
        s_kk[i] = f.kk[i];
        if (kRowsInLds && surf) {
            s_dl[i] = f.dlo[i];
            s_dh[i] = f.dhi[i];
        }
    }
    // entry e of the low (hi = false) or high plane's derivative row
    auto drow = [&](bool hi, int e) -> float2 {
        if constexpr (kRowsInLds) {
            return hi ? s_dh[e] : s_dl[e];
        } else {
            const float2 r = hi ? f.dhi[e] : f.dlo[e];
            return r;
        }
    };

    {
        const TileGeo geo = tile_geo<N, P, AXIS, SEG>(f, tile, pA, activeA);
        float2 raw[N1];
        load_tile<N, N1, N2, SEG, NTL && AXIS == 2>(psi, geo, n2, raw);
        // the y pass's epilogue operand (L from the x pass), the same elements
        // the epilogue writes, read by the thread that writes them.  Issued
        // once stage A is done, the field loads have the memory system to
        // themselves and L's latency still hides behind stage B and the
        // inverse stage A (issued with the field loads it cost 2-7 %); the
        // short pencils of segmented passes take it with the field loads
        // (the other way round there cost 2-3 %)
        float2 Lin[N1];
        auto load_L = [&]() {
            if constexpr (AXIS == 1) {
                const int C = SEG ? f.seg_core : N;
                const int H = SEG ? f.seg_halo : 0;
                unroll<N1>([&](auto i) {
                    constexpr int n1 = decltype(i)::value;
                    const int e = n2 + N2 * n1;
                    Lin[n1] = make_float2(0.f, 0.f);
                    if (geo.valid && e < N && (!SEG || (e >= H && e < H + C)))
                        Lin[n1] = f.L[geo.base + (int64_t)e * geo.estride];
                });
            }
        };
        if constexpr (SEG) load_L();
        GMEM const float* __restrict__ wloc = f.wloc;
        const int plane_lo = f.plane_lo, plane_hi = f.plane_hi;
        float2 v[N1];
        float2 plo = make_float2(0.f, 0.f), phi = plo;
        unroll<N1>([&](auto i) {
            constexpr int n1 = decltype(i)::value;
            const int e = n2 + N2 * n1;
            float2 x = raw[n1];
            if constexpr (SEG) x = cscale(x, e < N ? wloc[e] : 0.f);
            v[n1] = x;
        });
        // plane values: read directly by the thread that owns the element
        // (planes lie in a core, where the halo weight is 1)
        if (!ADJ && surf && geo.valid) {
            if (n2 == plane_lo % N2 && geo.seg == f.seg_plane0) plo = psi[geo.base + (int64_t)plane_lo * geo.estride];
            if (n2 == plane_hi % N2 && geo.seg == f.seg_plane1) phi = psi[geo.base + (int64_t)plane_hi * geo.estride];
        }
        __syncthreads();  // tables staged

        // spectral normal derivative on the two planes: partial dot products
        float2 dlo = make_float2(0.f, 0.f), dhi = dlo;
        if (!ADJ && surf) {
            unroll<N1>([&](auto i) {
                constexpr int n1 = decltype(i)::value;
                const int e = n2 + N2 * n1;
                if (e < N) {
                    dlo = cadd(dlo, cmul(drow(false, e), v[n1]));
                    dhi = cadd(dhi, cmul(drow(true, e), v[n1]));
                }
            });
        }

        // ---- forward: stage A (N1-point DFTs), twiddle, exchange ----
        dft<N1, -1>(v);
        if (activeA) {
            unroll<N1>([&](auto i) {
                constexpr int k1 = decltype(i)::value;
                float2 x = v[k1];
                if constexpr (k1 != 0) x = cmul(x, s_tw[n2 * k1]);
                ex[pA * STRIDE + k1 * ROW + n2] = x;
            });
        }
        // the values now live in LDS: clear the registers, so that threads idle
        // in stage A (which skip the reload below) do not keep them alive
        // through stage B
        unroll<N1>([&](auto i) { v[decltype(i)::value] = make_float2(0.f, 0.f); });
        if constexpr (!SEG) load_L();

        __syncthreads();

        // ---- stage B: N2-point DFT, kbar^2, inverse N2-point DFT ----
        if constexpr (M1 == 0) {
            if (t < P * N1) {
                // consecutive lanes on consecutive pencils (odd LDS stride) on
                // every axis: stage B touches LDS only
                const int pB = t % P;
                const int k1 = t / P;
                float2 u[N2];
                unroll<N2>([&](auto i) { u[decltype(i)::value] = ex[pB * STRIDE + k1 * ROW + decltype(i)::value]; });
                dft<N2, -1>(u);
                unroll<N2>([&](auto i) {
                    constexpr int k2 = decltype(i)::value;
                    u[k2] = cscale(u[k2], s_kk[k1 + N1 * k2]);
                });
                dft<N2, 1>(u);
                unroll<N2>([&](auto i) {
                    constexpr int nn = decltype(i)::value;
                    float2 x = u[nn];
                    if constexpr (nn != 0) x = cmulc(x, s_tw[nn * k1]);
                    ex[pB * STRIDE + k1 * ROW + nn] = x;
                });
            }
            __syncthreads();
        } else {
            // n2 = m2 + M2 m1, k2 = j1 + M1 j2: the N2-point DFT of row k1 is
            // M1-point DFTs over m1 (B1), the twiddle w_N2^{m2 j1}, and M2-point
            // DFTs over m2 (B2).  B1 works on the pairs (k1, m2) and writes
            // output j1 to slot m2 + M2 j1 of the row, so B2's inputs for
            // (k1, j1) are the M2 consecutive slots from M2 j1.
            constexpr int M2 = N2 / M1;
            static_assert(M1 * M2 == N2 && N1 % M1 == 0 && N1 % M2 == 0, "stage-B split");
            constexpr int R1 = N1 / M1;  // B1 pairs per thread
            constexpr int R2 = N1 / M2;  // B2 pairs per thread
            if (activeA) {
                unroll<R1>([&](auto ri) {
                    const int q = n2 + N2 * decltype(ri)::value;
                    const int k1 = q / M2, m2 = q - (q / M2) * M2;
                    float2* row = &ex[pA * STRIDE + k1 * ROW + m2];
                    float2 w[M1];
                    unroll<M1>([&](auto i) { w[decltype(i)::value] = row[M2 * decltype(i)::value]; });
                    dft<M1, -1>(w);
                    unroll<M1>([&](auto i) {
                        constexpr int j1 = decltype(i)::value;
                        float2 x = w[j1];
                        if constexpr (j1 != 0) x = cmul(x, s_tw[N1 * m2 * j1]);
                        row[M2 * j1] = x;
                    });
                });
            }
            __syncthreads();
            if (activeA) {
                unroll<R2>([&](auto ri) {
                    const int q = n2 + N2 * decltype(ri)::value;
                    const int k1 = q / M1, j1 = q - (q / M1) * M1;
                    float2* row = &ex[pA * STRIDE + k1 * ROW + M2 * j1];
                    float2 u[M2];
                    unroll<M2>([&](auto i) { u[decltype(i)::value] = row[decltype(i)::value]; });
                    dft<M2, -1>(u);
                    unroll<M2>([&](auto i) {
                        constexpr int j2 = decltype(i)::value;
                        u[j2] = cscale(u[j2], s_kk[k1 + N1 * (j1 + M1 * j2)]);
                    });
                    dft<M2, 1>(u);
                    unroll<M2>([&](auto i) { row[decltype(i)::value] = u[decltype(i)::value]; });
                });
            }
            __syncthreads();
            if (activeA) {
                unroll<R1>([&](auto ri) {
                    const int q = n2 + N2 * decltype(ri)::value;
                    const int k1 = q / M2, m2 = q - (q / M2) * M2;
                    float2* row = &ex[pA * STRIDE + k1 * ROW + m2];
                    float2 w[M1];
                    unroll<M1>([&](auto i) {
                        constexpr int j1 = decltype(i)::value;
                        float2 x = row[M2 * j1];
                        if constexpr (j1 != 0) x = cmulc(x, s_tw[N1 * m2 * j1]);
                        w[j1] = x;
                    });
                    dft<M1, 1>(w);
                    // back in slot n2 = m2 + M2 m1, with stage A's inverse twiddle
                    unroll<M1>([&](auto i) {
                        constexpr int m1 = decltype(i)::value;
                        float2 x = w[m1];
                        x = cmulc(x, s_tw[(m2 + M2 * m1) * k1]);
                        row[M2 * m1] = x;
                    });
                });
            }
            __syncthreads();
        }

        // ---- inverse: stage A ----
        if (activeA) {
            unroll<N1>([&](auto i) { v[decltype(i)::value] = ex[pA * STRIDE + decltype(i)::value * ROW + n2]; });
        }
        dft<N1, 1>(v);

        // surface point of this pencil on the planes normal to the axis
        int64_t pt;
        if constexpr (AXIS == 0) pt = (int64_t)tile * P + pA;
        else pt = geo.tx * P + pA + (int64_t)f.nx * geo.tq;

        // ---- adjoint steps: the surface terms injected along this pencil,
        // c (plane values on the planes + derivative rows times the derivative
        // parts), c = i w_m from the step table ----
        if constexpr (ADJ) {
            if (surf) {
                float2 hpl = make_float2(0.f, 0.f), hdl = hpl, hph = hpl, hdh = hpl;
                if (geo.valid) {
                    const double2 cw = f.w_tab[nstep];
                    const float2 cinj = make_float2((float)cw.x, (float)cw.y);
                    hpl = cmul(cinj, f.inj_lo_p[pt]);
                    hdl = cmul(cinj, f.inj_lo_d[pt]);
                    hph = cmul(cinj, f.inj_hi_p[pt]);
                    hdh = cmul(cinj, f.inj_hi_d[pt]);
                }
                unroll<N1>([&](auto i) {
                    constexpr int n1 = decltype(i)::value;
                    const int e = n2 + N2 * n1;
                    if (e < N) {
                        float2 x = cadd(cmul(drow(false, e), hdl), cmul(drow(true, e), hdh));
                        if (e == plane_lo) x = cadd(x, hpl);
                        if (e == plane_hi) x = cadd(x, hph);
                        v[n1] = cadd(v[n1], x);
                    }
                });
            }
        }

        // ---- epilogue (only core elements are written) ----
        const int C = SEG ? f.seg_core : N;
        const int H = SEG ? f.seg_halo : 0;
        GMEM float2* __restrict__ Lbuf = f.L;
        if (geo.valid) {
            if constexpr (AXIS == 0 && POTX) {
                // the potential term 2 dtau V / E0 psi^n of the row's cells when V's
                // box covers few rows: rows off the box store the kinetic term alone,
                // the others read psi^n again (the tile was just read, so this hits
                // the cache) rather than hold it in registers through the transforms
                const int64_t row = ((int64_t)tile * P + pA) / (SEG ? f.nseg : 1);
                const int z = (int)((unsigned)row / (unsigned)f.ny), y = (int)row - z * f.ny;
                const bool brow = (unsigned)(y - f.vlo1) < (unsigned)f.vn1 && (unsigned)(z - f.vlo2) < (unsigned)f.vn2;
                if (!brow) {
                    unroll<N1>([&](auto i) {
                        constexpr int n1 = decltype(i)::value;
                        const int e = n2 + N2 * n1;
                        if (e < N && (!SEG || (e >= H && e < H + C))) Lbuf[geo.base + e] = v[n1];
                    });
                } else {
                    // every load first (the box value through a clamped index), then
                    // the products and stores, so the loads overlap
                    const int64_t vrow = ((int64_t)(z - f.vlo2) * f.vn1 + (y - f.vlo1)) * f.vn0 - f.vlo0;
                    float2 pv[N1];
                    float vv[N1];
                    unroll<N1>([&](auto i) {
                        constexpr int n1 = decltype(i)::value;
                        const int e = n2 + N2 * n1;
                        const int x = geo.g0 + e;
                        const bool own = e < N && (!SEG || (e >= H && e < H + C));
                        const bool inb = own && (unsigned)(x - f.vlo0) < (unsigned)f.vn0;
                        pv[n1] = make_float2(0.f, 0.f);
                        if (own) pv[n1] = psi[geo.base + e];
                        const float b = f.vbox[inb ? vrow + x : 0];
                        vv[n1] = inb ? b : 0.f;
                    });
                    unroll<N1>([&](auto i) {
                        constexpr int n1 = decltype(i)::value;
                        const int e = n2 + N2 * n1;
                        if (e < N && (!SEG || (e >= H && e < H + C)))
                            Lbuf[geo.base + e] = cadd(v[n1], cscale(pv[n1], vv[n1]));
                    });
                }
            } else if constexpr (AXIS == 0) {
                unroll<N1>([&](auto i) {
                    constexpr int n1 = decltype(i)::value;
                    const int e = n2 + N2 * n1;
                    if (e < N && (!SEG || (e >= H && e < H + C))) Lbuf[geo.base + e] = v[n1];
                });
            } else if constexpr (AXIS == 1) {
                unroll<N1>([&](auto i) {
                    constexpr int n1 = decltype(i)::value;
                    const int e = n2 + N2 * n1;
                    if (e < N && (!SEG || (e >= H && e < H + C))) {
                        const int64_t ad = geo.base + (int64_t)e * geo.estride;
                        Lbuf[ad] = cadd(Lin[n1], v[n1]);
                    }
                });
            } else {
                GMEM const float* __restrict__ t_gam = f.gam;
                GMEM const float4* __restrict__ t_zd = f.zd;
                const int px = geo.px, py = geo.py;
                const float2 Zx = f.zt_x[px], Dx = f.dz_x[px];
                const float2 Zy = f.zt_y[py], Dy = f.dz_y[py];
                const float2 SA = cadd(cmul(Dx, Zy), cmul(Zx, Dy));  // source terms of axes x, y
                const float2 SB = cmul(Zx, Zy);                      // multiplies the z-axis term
                const float gxy = f.gam_x[px] * f.gam_y[py];
                float2 sigma = make_float2(0.f, 0.f);
                if constexpr (!ADJ) sigma = f.sigma_tab[nstep];
                GMEM const float2* __restrict__ fwd = nullptr;
                GMEM float2* __restrict__ stash = nullptr;
                if constexpr (ADJ) fwd = gmem(f.fwd_tab[nstep]);
                else if (f.stash_tab) stash = gmem(f.stash_tab[nstep]);
                // the potential term 2 dtau (V / E0 + sum_a w_a) psi^n: V is read on
                // the pencils that cross its box only (the box value through a
                // clamped index, so the loads of a pencil are not branched apart)
                const bool bpen = (unsigned)(px - f.vlo0) < (unsigned)f.vn0 && (unsigned)(py - f.vlo1) < (unsigned)f.vn1;
                const int64_t vcol = (int64_t)(py - f.vlo1) * f.vn0 + (px - f.vlo0);
                const int64_t vplane = (int64_t)f.vn0 * f.vn1;
                GMEM const float* __restrict__ wr0 = f.wr0;
                const float wxy = wr0 ? wr0[px] + f.wr1[py] : 0.f;
                float vv[N1];
                if (!POTX && (bpen || wr0)) {
                    unroll<N1>([&](auto i) {
                        constexpr int n1 = decltype(i)::value;
                        const int z = geo.g0 + n2 + N2 * n1;
                        const bool inb = bpen && (unsigned)(z - f.vlo2) < (unsigned)f.vn2;
                        const float b = f.vbox[inb ? vcol + (int64_t)(z - f.vlo2) * vplane : 0];
                        vv[n1] = (inb ? b : 0.f) + (wr0 && z >= 0 && z < f.nz ? wxy + f.wr2[z] : 0.f);
                    });
                } else {
                    unroll<N1>([&](auto i) { vv[decltype(i)::value] = 0.f; });
                }
                unroll<N1>([&](auto i) {
                    constexpr int n1 = decltype(i)::value;
                    const int e = n2 + N2 * n1;
                    if (e < N && (!SEG || (e >= H && e < H + C))) {
                        const int z = geo.g0 + e;
                        const int64_t ad = geo.base + (int64_t)e * geo.estride;
                        const float2 Lt = cadd(load_last<NTL>(Lbuf + ad), v[n1]);
                        const float2 po = load_last<NTL>(psi_old + ad);
                        float2 q = Lt;
                        if constexpr (!POTX) q = cadd(q, cscale(raw[n1], vv[n1]));
                        if constexpr (!ADJ) {
                            const float4 zd = t_zd[z];
                            const float2 s = cadd(cmul(SA, make_float2(zd.x, zd.y)), cmul(SB, make_float2(zd.z, zd.w)));
                            q = cadd(q, cmul(sigma, s));
                        }
                        const float g = gxy * t_gam[z];
                        // psi^{n+1} = Gamma (psi^{n-1} - i q)
                        const float2 nv = make_float2(g * (po.x + q.y), g * (po.y - q.x));
                        psi_old[ad] = nv;
                        if (stash) stash[ad] = nv;
                        if constexpr (ADJ) {
                            // Im(chi^m psi^{m-1})
                            const float2 fv = fwd[ad];
                            f.grad[ad] += nv.x * fv.y + nv.y * fv.x;
                        }
                    }
                });
            }
        }

        // ---- surface DFT: reduce the per-thread partials, accumulate in FP64 ----
        if (!ADJ && surf) {
            __syncthreads();  // every thread has read its exchange slots
            if (activeA) {
                float2* r = &ex[pA * STRIDE + n2 * 4];
                r[0] = plo;
                r[1] = phi;
                r[2] = dlo;
                r[3] = dhi;
            }
            __syncthreads();
            if (t < P * 4) {
                const int p = t >> 2;
                const int q = t & 3;
                const int side = q & 1;
                const int segp = side ? f.seg_plane1 : f.seg_plane0;
                const int nseg = SEG ? f.nseg : 1;
                int64_t spt = -1;
                if constexpr (AXIS == 0) {
                    const int64_t qq = (int64_t)tile * P + p;
                    if (qq < (int64_t)f.ny * f.nz * nseg && (int)(qq % nseg) == segp) spt = qq / nseg;
                } else {
                    const int x = geo.tx * P + p;
                    if (x < f.nx && geo.tq % nseg == segp) spt = x + (int64_t)f.nx * (geo.tq / nseg);
                }
                if (spt >= 0 && f.bstage) {
                    // pulsed runs: stage the plane value of this step of the group
                    float2 s = make_float2(0.f, 0.f);
                    for (int m = 0; m < N2; ++m) s = cadd(s, ex[p * STRIDE + m * 4 + q]);
                    f.bstage[((int64_t)(koff * 2 + side) * 2 + (q >> 1)) * f.points + spt] = s;
                } else if (spt >= 0) {
                    float2 s = make_float2(0.f, 0.f);
                    for (int m = 0; m < N2; ++m) s = cadd(s, ex[p * STRIDE + m * 4 + q]);
                    const double re = (double)s.x, im = (double)s.y;
                    const double2 w = f.w_tab[nstep];
                    const double zr = w.x * re - w.y * im;
                    const double zi = w.x * im + w.y * re;
                    const int field = (q >> 1) * 2;
                    const int64_t points = f.points;
                    GMEM double2* __restrict__ S = f.acc + (int64_t)(side * 4 + field) * points + spt;
                    GMEM double2* __restrict__ Cc = f.acc + (int64_t)(side * 4 + field + 1) * points + spt;
                    double2 sv = *S, cv = *Cc;
                    neumaier(sv.x, cv.x, zr);
                    neumaier(sv.y, cv.y, zi);
                    *S = sv;
                    *Cc = cv;
                }
            }
        }
    }
}

using LaunchFn = hipError_t (*)(int axis, const PassArgs& single, const PassArgs* descs, const int* off, int ninst,
                                int tiles, int koff, hipStream_t stream);

template <int N, int N1, int N2, int M1, int P, int AXIS, bool SEG, bool MULTI, bool ADJ, bool POTX = false,
          bool NTL = false>
hipError_t launch_kernel(const PassArgs& single, const PassArgs* descs, const int* off, int ninst, int tiles,
                         int koff, hipStream_t stream) {
    constexpr int threads = P * (N1 > N2 ? N1 : N2);
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((pass_kernel<N, N1, N2, M1, P, AXIS, SEG, MULTI, ADJ, POTX, NTL>), dim3(tiles), dim3(threads), 0,
                       stream, single, descs, off, ninst, koff);
    return hipGetLastError();
}

// the z pass, with or without non-temporal loads of its last-use operands
template <int N, int N1, int N2, int M1, int P, bool SEG, bool MULTI, bool POTX>
hipError_t launch_z(const PassArgs& single, const PassArgs* descs, const int* off, int ninst, int tiles, int koff,
                    hipStream_t stream) {
    if (single.nt)
        return launch_kernel<N, N1, N2, M1, P, 2, SEG, MULTI, false, POTX, true>(single, descs, off, ninst, tiles, koff,
                                                                                  stream);
    return launch_kernel<N, N1, N2, M1, P, 2, SEG, MULTI, false, POTX, false>(single, descs, off, ninst, tiles, koff,
                                                                               stream);
}

template <int N, int N1, int N2, int M1, int P, bool SEG>
static hipError_t launch_shape(int axis, const PassArgs& single, const PassArgs* descs, const int* off, int ninst,
                               int tiles, int koff, hipStream_t stream) {
    if (ninst == 0) {
        // unsegmented axes may take the potential in the x pass
        if (!SEG && single.potx) {
            if (axis == 0) return launch_kernel<N, N1, N2, M1, P, 0, false, false, false, true>(single, descs, off, 0, tiles, koff, stream);
            if (axis == 2) return launch_z<N, N1, N2, M1, P, false, false, true>(single, descs, off, 0, tiles, koff, stream);
        }
        if (axis == 0) return launch_kernel<N, N1, N2, M1, P, 0, SEG, false, false>(single, descs, off, 0, tiles, koff, stream);
        if (axis == 1) return launch_kernel<N, N1, N2, M1, P, 1, SEG, false, false>(single, descs, off, 0, tiles, koff, stream);
        return launch_z<N, N1, N2, M1, P, SEG, false, false>(single, descs, off, 0, tiles, koff, stream);
    }
    if (!SEG && single.potx) {
        if (axis == 0) return launch_kernel<N, N1, N2, M1, P, 0, false, true, false, true>(single, descs, off, ninst, tiles, koff, stream);
        if (axis == 2) return launch_z<N, N1, N2, M1, P, false, true, true>(single, descs, off, ninst, tiles, koff, stream);
    }
    if (axis == 0) return launch_kernel<N, N1, N2, M1, P, 0, SEG, true, false>(single, descs, off, ninst, tiles, koff, stream);
    if (axis == 1) return launch_kernel<N, N1, N2, M1, P, 1, SEG, true, false>(single, descs, off, ninst, tiles, koff, stream);
    return launch_z<N, N1, N2, M1, P, SEG, true, false>(single, descs, off, ninst, tiles, koff, stream);
}

template <int N, int N1, int N2, int M1, int P>
static hipError_t launch_adjoint_shape(int axis, const PassArgs& a, int koff, hipStream_t stream) {
    if (axis == 0) return launch_kernel<N, N1, N2, M1, P, 0, false, false, true>(a, nullptr, nullptr, 0, a.tiles, koff, stream);
    if (axis == 1) return launch_kernel<N, N1, N2, M1, P, 1, false, false, true>(a, nullptr, nullptr, 0, a.tiles, koff, stream);
    return launch_kernel<N, N1, N2, M1, P, 2, false, false, true>(a, nullptr, nullptr, 0, a.tiles, koff, stream);
}

using AdjFn = hipError_t (*)(int axis, const PassArgs& a, int koff, hipStream_t stream);

template <int S, int N, int N1, int N2, int M1, int P>
hipError_t launch_segmented_shape(int axis, const PassArgs& single, const PassArgs* descs, const int* off, int ninst,
                                  int tiles, int koff, hipStream_t stream) {
    if constexpr (S != 0) return launch_shape<N, N1, N2, M1, P, true>(axis, single, descs, off, ninst, tiles, koff, stream);
    else return hipErrorInvalidValue;
}

// entry points of one compiled shape, named after it
#define PSTD_FN(kind, N_, A_, B_, M_, P_) pass_##kind##_##N_##_##A_##_##B_##_##M_##_##P_
#define PSTD_DECLARE_SHAPE(N_, A_, B_, M_, P_, S_, PART_)                                                         \
    hipError_t PSTD_FN(plain, N_, A_, B_, M_, P_)(int, const PassArgs&, const PassArgs*, const int*, int, int, int, \
                                                 hipStream_t);                                                   \
    hipError_t PSTD_FN(seg, N_, A_, B_, M_, P_)(int, const PassArgs&, const PassArgs*, const int*, int, int, int,   \
                                               hipStream_t);                                                     \
    hipError_t PSTD_FN(adj, N_, A_, B_, M_, P_)(int, const PassArgs&, int, hipStream_t);
#define PSTD_DEFINE_SHAPE(N_, A_, B_, M_, P_, S_)                                                                   \
    hipError_t PSTD_FN(plain, N_, A_, B_, M_, P_)(int axis, const PassArgs& single, const PassArgs* descs,            \
                                                 const int* off, int ninst, int tiles, int koff, hipStream_t stream) { \
        return launch_shape<N_, A_, B_, M_, P_, false>(axis, single, descs, off, ninst, tiles, koff, stream);          \
    }                                                                                                              \
    hipError_t PSTD_FN(seg, N_, A_, B_, M_, P_)(int axis, const PassArgs& single, const PassArgs* descs,              \
                                               const int* off, int ninst, int tiles, int koff, hipStream_t stream) {   \
        return launch_segmented_shape<S_, N_, A_, B_, M_, P_>(axis, single, descs, off, ninst, tiles, koff, stream);   \
    }                                                                                                              \
    hipError_t PSTD_FN(adj, N_, A_, B_, M_, P_)(int axis, const PassArgs& args, int koff, hipStream_t stream) {       \
        return launch_adjoint_shape<N_, A_, B_, M_, P_>(axis, args, koff, stream);                                    \
    }

}  // namespace pstd
