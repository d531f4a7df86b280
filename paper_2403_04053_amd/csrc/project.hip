// Near-to-distant-field projection over the virtual box (Section 3.2).
//
// All sums are FP64.  The phasors of each face plane are first brought to
// their 2D spectrum (the coefficients of the trigonometric interpolant of
// Eq. AnBottomPsi).  Then:
//
//  * far field: the cell formula of Eqs. bottomPsi_lm ... leftrightPsi_ln in
//    the limit of Eq. FDTDfarfieldapprox.  For a direction r_hat every cell
//    term factors into an in-plane b-part and c-part, so a face contributes
//    g_c(r_hat)^T [F_dpsi + i r_hat_a F_psi] g_b(r_hat): one complex GEMM
//    [directions x Nb] x [Nb x 2Nc] per face and a fused row-wise dot;
//  * Fresnel points: each sinc of the cell formula is expanded to 8th order
//    in its shift alpha = k d R_hat / 2, so the spectral double sum of a cell
//    becomes sum_pq alpha_b^p alpha_c^q Q_pq(cell); the Q tables are two
//    batched GEMMs per face and field, and the per-point work is a Horner
//    evaluation per cell with the exact distance R and exp(ikR)/R.
//
// Reduced units throughout (k = 1); the far-field amplitude is divided by k0
// at the end to return physical length units.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "project.hpp"

namespace pstd {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kOrder = 8;            // sinc expansion order
constexpr int kTerms = kOrder + 1;

__host__ __device__ inline int face_axis_b(int a) { return a == 0 ? 1 : 0; }
__host__ __device__ inline int face_axis_c(int a) { return a == 2 ? 1 : 2; }

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double dsinc(double x) { return fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sin(x) / x; }

// ---------------------------------------------------------------------------
// phasor finalisation
// ---------------------------------------------------------------------------

__global__ void finalize_kernel(const double2* __restrict__ acc, int side, int64_t points, double2 sv, double2 sd,
                                double2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= points) return;
    const double2* base = acc + (int64_t)side * 4 * points;
    const double2 s0 = base[i], c0 = base[points + i], s1 = base[2 * points + i], c1 = base[3 * points + i];
    const double ar = s0.x + c0.x, ai = s0.y + c0.y, br = s1.x + c1.x, bi = s1.y + c1.y;
    out[i] = make_double2(ar * sv.x - ai * sv.y, ar * sv.y + ai * sv.x);
    out[points + i] = make_double2(br * sd.x - bi * sd.y, br * sd.y + bi * sd.x);
}

// ---------------------------------------------------------------------------
// naive separable 2D DFT of a [Nc][Nb] plane (FP64, forward)
// ---------------------------------------------------------------------------

__global__ void dft_rows_kernel(const double2* __restrict__ x, double2* __restrict__ y, int Nb, int Nc,
                                const double2* __restrict__ twb) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)Nb * Nc) return;
    const int bp = (int)(id % Nb), c = (int)(id / Nb);
    double2 s = make_double2(0, 0);
    for (int b = 0; b < Nb; ++b) s = zadd(s, zmul(x[(int64_t)c * Nb + b], twb[(int)(((int64_t)b * bp) % Nb)]));
    y[id] = s;
}

__global__ void dft_cols_kernel(const double2* __restrict__ y, double2* __restrict__ z, int Nb, int Nc,
                                const double2* __restrict__ twc) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)Nb * Nc) return;
    const int bp = (int)(id % Nb), cp = (int)(id / Nb);
    double2 s = make_double2(0, 0);
    for (int c = 0; c < Nc; ++c) s = zadd(s, zmul(y[(int64_t)c * Nb + bp], twc[(int)(((int64_t)c * cp) % Nc)]));
    z[id] = s;
}

// ---------------------------------------------------------------------------
// batched complex GEMM on the FP64 matrix cores, row-major:
// C[i][j] = sum_k A[i][k] B[k][j]
//
// v_mfma_f64_16x16x4f64 takes, per lane l, A[i][k] with i = l % 16, k = l / 16
// and B[k][j] with j = l % 16, k = l / 16, and leaves D[i][j] in register r
// of lane l for i = 4 r + l / 16, j = l % 16.  A complex product is four real
// ones: re += Ar Br - Ai Bi, im += Ar Bi + Ai Br.  A workgroup (4 waves)
// computes a 64 x 64 tile, each wave 32 x 32 (2 x 2 MFMA tiles), from
// 16-deep slices of A and B staged in LDS.
// ---------------------------------------------------------------------------

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int ZT = 64;   // output tile edge
constexpr int ZK = 16;   // K slice

__global__ __launch_bounds__(256) void zgemm_kernel(int M, int N, int K, const double2* __restrict__ A, int64_t lda,
                                                    int64_t sA, const double2* __restrict__ B, int64_t ldb, int64_t sB,
                                                    double2* __restrict__ C, int64_t ldc, int64_t sC) {
    __shared__ double2 As[ZT][ZK + 1];
    __shared__ double2 Bs[ZK][ZT + 1];
    const int bz = blockIdx.z;
    A += bz * sA;
    B += bz * sB;
    C += bz * sC;
    const int i0 = blockIdx.y * ZT, j0 = blockIdx.x * ZT;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    v4d re[2][2], im[2][2];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            re[u][v] = v4d{0, 0, 0, 0};
            im[u][v] = v4d{0, 0, 0, 0};
        }
    for (int k0 = 0; k0 < K; k0 += ZK) {
        for (int e = t; e < ZT * ZK; e += 256) {
            const int r = e / ZK, c = e % ZK;
            const int gi = i0 + r, gk = k0 + c;
            As[r][c] = (gi < M && gk < K) ? A[(int64_t)gi * lda + gk] : make_double2(0, 0);
        }
        for (int e = t; e < ZK * ZT; e += 256) {
            const int r = e / ZT, c = e % ZT;
            const int gk = k0 + r, gj = j0 + c;
            Bs[r][c] = (gk < K && gj < N) ? B[(int64_t)gk * ldb + gj] : make_double2(0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < ZK; ks += 4) {
            double2 a[2], b[2];
            for (int u = 0; u < 2; ++u) a[u] = As[wi + u * 16 + li][ks + lk];
            for (int v = 0; v < 2; ++v) b[v] = Bs[ks + lk][wj + v * 16 + li];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[v].x, re[u][v], 0, 0, 0);
                    re[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].y, b[v].y, re[u][v], 0, 0, 0);
                    im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[v].y, im[u][v], 0, 0, 0);
                    im[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, b[v].x, im[u][v], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + wi + u * 16 + 4 * r + lk, gj = j0 + wj + v * 16 + li;
                if (gi < M && gj < N) C[(int64_t)gi * ldc + gj] = make_double2(re[u][v][r], im[u][v][r]);
            }
}

hipError_t zgemm(int M, int N, int K, const double2* A, int64_t lda, int64_t sA, const double2* B, int64_t ldb,
                 int64_t sB, double2* C, int64_t ldc, int64_t sC, int batch, hipStream_t stream) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    dim3 grid((N + ZT - 1) / ZT, (M + ZT - 1) / ZT, batch);
    hipLaunchKernelGGL(zgemm_kernel, grid, dim3(256), 0, stream, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// far field
// ---------------------------------------------------------------------------

// g(b') = (-1)^b' sinc(pi b'/N - d r/2) sum_{l=lo}^{hi-1} exp(i (2 pi b'/(N d) - r) x_l),
// x_l = (l - N/2 + 1/2) d: the closed form of the geometric sum is used.
__global__ void farfield_factor_kernel(const double3* __restrict__ dirs, int64_t nd, int comp, int N, double d,
                                       int lo, int hi, double2* __restrict__ G) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nd * N) return;
    const int m = (int)(id % N);
    const int64_t di = id / N;
    const double3 rh = dirs[di];
    const double r = comp == 0 ? rh.x : comp == 1 ? rh.y : rh.z;
    const int bp = m < N / 2 ? m : m - N;
    const double beta = 2.0 * kPi * bp / (N * d) - r;
    const int M = hi - lo;
    const double theta = beta * d / 2.0;
    const double mag = (double)M * dsinc(M * theta) / dsinc(theta) * dsinc(kPi * bp / N - d * r / 2.0) *
                       ((bp & 1) ? -1.0 : 1.0);
    const double ph = beta * d * (lo - N / 2 + 0.5 * M);
    double sn, cs;
    sincos(ph, &sn, &cs);
    G[id] = make_double2(mag * cs, mag * sn);
}

// Mt[b'][j] = F_dpsi[j][b'] (j < Nc), F_psi[j - Nc][b'] (j >= Nc)
__global__ void stack_transpose_kernel(const double2* __restrict__ Fp, const double2* __restrict__ Fd, int Nb, int Nc,
                                       double2* __restrict__ Mt) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)Nb * 2 * Nc) return;
    const int j = (int)(id % (2 * Nc));
    const int bp = (int)(id / (2 * Nc));
    Mt[id] = j < Nc ? Fd[(int64_t)j * Nb + bp] : Fp[(int64_t)(j - Nc) * Nb + bp];
}

// f[d] += pref exp(-i r_a x_a) sum_c' Gc[d][c'] (T[d][c'] + i r_a T[d][Nc + c'])
// One wave per direction: the lanes read consecutive c' (coalesced rows of T
// and Gc) and the partial sums are reduced across the wave.
constexpr int kDotWaves = 4;

__global__ __launch_bounds__(64 * kDotWaves) void farfield_dot_kernel(const double3* __restrict__ dirs, int64_t nd,
                                                                      int comp_a, double xa, double pref,
                                                                      const double2* __restrict__ Gc,
                                                                      const double2* __restrict__ T, int Nc,
                                                                      double2* __restrict__ f) {
    const int lane = threadIdx.x & 63;
    const int64_t d = (int64_t)blockIdx.x * kDotWaves + (threadIdx.x >> 6);
    if (d >= nd) return;  // whole wave
    const double3 rh = dirs[d];
    const double ra = comp_a == 0 ? rh.x : comp_a == 1 ? rh.y : rh.z;
    double sx = 0, sy = 0;
    const double2* t = T + d * 2 * Nc;
    const double2* g = Gc + d * Nc;
    for (int c = lane; c < Nc; c += 64) {
        const double2 a = t[c], b = t[Nc + c];
        // a + i ra b
        const double2 m = make_double2(a.x - ra * b.y, a.y + ra * b.x);
        const double2 p = zmul(g[c], m);
        sx += p.x;
        sy += p.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_down(sx, o, 64);
        sy += __shfl_down(sy, o, 64);
    }
    if (lane == 0) {
        double sn, cs;
        sincos(-ra * xa, &sn, &cs);
        const double2 r = zmul(make_double2(sx, sy), make_double2(pref * cs, pref * sn));
        f[d] = zadd(f[d], r);
    }
}

// ---------------------------------------------------------------------------
// Fresnel points
// ---------------------------------------------------------------------------

constexpr int kNearThreads = 128;
constexpr int kNearPoints = 4;  // observation points per thread in near_kernel
constexpr int kCellChunk = 8;

struct FaceGeo {
    int a, b, c;
    int lo_b, lo_c, L, M;     // cell ranges
    double db, dc, xa;        // reduced spacings, face coordinate
    double xb0, xc0;          // first cell-centre coordinates
    double pref;
};

// Q layout: [cell][field(0 psi, 1 dpsi)][p][q]
// One thread per point; workgroup row blockIdx.y sums the cells
// [y * cells_per_split, (y + 1) * cells_per_split), so that few points still
// fill the chip.  Each row writes its partial sum (times the face prefactor)
// to part[y * n_obs + point]; add_splits_kernel adds the rows in order.
// K observation points per thread, kNearThreads apart (coalesced loads and
// stores): each coefficient read from LDS serves K points, which takes the
// kernel off the LDS read rate (one 16-byte broadcast per two FP64 FMAs
// with one point per thread).  Each point's sums run in the same order as
// with one point per thread.
template <int K>
__global__ __launch_bounds__(kNearThreads) void near_kernel(const double3* __restrict__ obs, int64_t n_obs, double k0,
                                                            FaceGeo g, const double2* __restrict__ Q,
                                                            int64_t cells_per_split, double2* __restrict__ part) {
    __shared__ double2 sq[kCellChunk * 2 * kTerms * kTerms];
    bool live[K];
    bool any_live = false;
    double Ra[K], rb_[K], rc_[K];  // point in the face frame (normal, b, c)
    double2 acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t pi = ((int64_t)blockIdx.x * K + k) * kNearThreads + threadIdx.x;
        live[k] = pi < n_obs;
        any_live |= live[k];
        // an idle slot gets a point one unit off the face, so that its
        // (discarded) sums stay finite
        double ra = g.xa + 1.0, rb = 0, rc = 0;
        if (live[k]) {
            const double3 o = obs[pi];
            const double x = o.x * k0, y = o.y * k0, z = o.z * k0;
            ra = g.a == 0 ? x : g.a == 1 ? y : z;
            rb = g.b == 0 ? x : g.b == 1 ? y : z;
            rc = g.c == 0 ? x : g.c == 1 ? y : z;
        }
        Ra[k] = ra - g.xa;
        rb_[k] = rb;
        rc_[k] = rc;
        acc[k] = make_double2(0, 0);
    }
    const int64_t ncell = (int64_t)g.L * g.M;
    const int64_t c_lo = (int64_t)blockIdx.y * cells_per_split;
    const int64_t c_hi = min<int64_t>(ncell, c_lo + cells_per_split);
    constexpr int per_cell = 2 * kTerms * kTerms;
    for (int64_t c0 = c_lo; c0 < c_hi; c0 += kCellChunk) {
        const int nc = (int)min<int64_t>(kCellChunk, c_hi - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < nc * per_cell; e += kNearThreads) sq[e] = Q[c0 * per_cell + e];
        __syncthreads();
        if (!any_live) continue;
        for (int ci = 0; ci < nc; ++ci) {
            const int64_t cell = c0 + ci;
            const int m = (int)(cell / g.L), l = (int)(cell % g.L);
            double Rn[K], inv[K], ab[K], ac[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double Rb = rb_[k] - (g.xb0 + l * g.db);
                const double Rc = rc_[k] - (g.xc0 + m * g.dc);
                const double R2 = Ra[k] * Ra[k] + Rb * Rb + Rc * Rc;
                Rn[k] = sqrt(R2);
                inv[k] = 1.0 / Rn[k];
                ab[k] = g.db * Rb * inv[k] * 0.5;
                ac[k] = g.dc * Rc * inv[k] * 0.5;
            }
            const double2* q = &sq[ci * per_cell];
            double2 S0[K], S1[K];
#pragma unroll 1
            for (int fld = 0; fld < 2; ++fld) {
                double2 outer[K];
#pragma unroll
                for (int k = 0; k < K; ++k) outer[k] = make_double2(0, 0);
#pragma unroll 1
                for (int p = kOrder; p >= 0; --p) {
                    double2 inner[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) inner[k] = make_double2(0, 0);
                    const double2* row = q + (fld * kTerms + p) * kTerms;
#pragma unroll
                    for (int qq = kOrder; qq >= 0; --qq) {
                        const double2 cq = row[qq];
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            inner[k].x = inner[k].x * ac[k] + cq.x;
                            inner[k].y = inner[k].y * ac[k] + cq.y;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        outer[k].x = outer[k].x * ab[k] + inner[k].x;
                        outer[k].y = outer[k].y * ab[k] + inner[k].y;
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (fld == 0) S0[k] = outer[k];
                    else S1[k] = outer[k];
                }
            }
            // e^{iR}/R (S_dpsi + (i - 1/R) (R_a/R) S_psi)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double ra = Ra[k] * inv[k];
                const double2 coef = make_double2(-inv[k] * ra, ra);
                const double2 inner = zadd(S1[k], zmul(coef, S0[k]));
                double sn, cs;
                sincos(Rn[k], &sn, &cs);
                acc[k] = zadd(acc[k], zmul(make_double2(cs * inv[k], sn * inv[k]), inner));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t pi = ((int64_t)blockIdx.x * K + k) * kNearThreads + threadIdx.x;
        if (live[k]) part[(int64_t)blockIdx.y * n_obs + pi] = make_double2(acc[k].x * g.pref, acc[k].y * g.pref);
    }
}

// out[i] (+)= sum over the split rows k = 0, 1, ... of part[k * n + i], in
// row order
__global__ void add_splits_kernel(const double2* __restrict__ part, int splits, int64_t n, bool accumulate,
                                  double2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = part[i];
    for (int k = 1; k < splits; ++k) acc = zadd(acc, part[(int64_t)k * n + i]);
    out[i] = accumulate ? zadd(out[i], acc) : acc;
}

// Adjoint of the per-point cell sums: for one cell and one p,
// Qbar[fld][p][q][cell] = sum_o conj(pref e^{iR}/R alpha_b^p alpha_c^q [coef]) g_o,
// coef = (i - 1/R) R_a / R for the psi field (fld 0), 1 for dpsi (fld 1).
constexpr int kAdjObsChunk = 256;
constexpr int kAdjP = 3;  // values of p per thread in near_adjoint_kernel

// Workgroup row blockIdx.y sums the points [y * obs_per_split, (y + 1) *
// obs_per_split) into its own copy of Qbar (Qbar + y * 2 kTerms^2 ncell);
// add_splits_kernel adds the copies in order.
template <int KP>
__global__ __launch_bounds__(128) void near_adjoint_kernel(const double3* __restrict__ obs, const double2* __restrict__ gv,
                                                           int64_t n_obs, double k0, FaceGeo g,
                                                           int64_t obs_per_split, double2* __restrict__ Qbar) {
    // one thread per (cell, block of KP consecutive p): the distance, the
    // square root and the sincos of a (cell, point) pair are taken once for
    // KP values of p; each (field, p, q) sum runs over the points in the same
    // order as with one p per thread
    constexpr int kBlocks = (kTerms + KP - 1) / KP;
    __shared__ double3 so[kAdjObsChunk];
    __shared__ double2 sg[kAdjObsChunk];
    const int64_t ncell = (int64_t)g.L * g.M;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = id < ncell * kBlocks;
    const int64_t cell = live ? id % ncell : 0;
    const int p0 = live ? (int)(id / ncell) * KP : 0;
    const int m = (int)(cell / g.L), l = (int)(cell % g.L);
    const double yb = g.xb0 + l * g.db, yc = g.xc0 + m * g.dc;
    double2 acc[KP][2][kTerms];
#pragma unroll
    for (int j = 0; j < KP; ++j)
        for (int f = 0; f < 2; ++f)
            for (int q = 0; q < kTerms; ++q) acc[j][f][q] = make_double2(0, 0);
    const int64_t o_lo = (int64_t)blockIdx.y * obs_per_split;
    const int64_t o_hi = min<int64_t>(n_obs, o_lo + obs_per_split);
    for (int64_t o0 = o_lo; o0 < o_hi; o0 += kAdjObsChunk) {
        const int no = (int)min<int64_t>(kAdjObsChunk, o_hi - o0);
        __syncthreads();
        for (int e = threadIdx.x; e < no; e += blockDim.x) {
            so[e] = obs[o0 + e];
            sg[e] = gv[o0 + e];
        }
        __syncthreads();
        if (!live) continue;
        for (int e = 0; e < no; ++e) {
            const double x = so[e].x * k0, y = so[e].y * k0, z = so[e].z * k0;
            const double Ra = (g.a == 0 ? x : g.a == 1 ? y : z) - g.xa;
            const double Rb = (g.b == 0 ? x : g.b == 1 ? y : z) - yb;
            const double Rc = (g.c == 0 ? x : g.c == 1 ? y : z) - yc;
            const double Rn = sqrt(Ra * Ra + Rb * Rb + Rc * Rc);
            const double inv = 1.0 / Rn;
            const double ab = g.db * Rb * inv * 0.5, ac = g.dc * Rc * inv * 0.5;
            double sn, cs;
            sincos(Rn, &sn, &cs);
            const double2 gg = sg[e];
            const double rr = Ra * inv;
            // alpha_b^p0 by the same product as with one p per thread
            double abp = 1.0;
            for (int t = 0; t < p0; ++t) abp *= ab;
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                // conj(pref e^{iR}/R alpha_b^p) g
                const double wr = g.pref * inv * abp;
                const double2 base = make_double2(wr * (cs * gg.x + sn * gg.y), wr * (cs * gg.y - sn * gg.x));
                // conj(coef) = (-i - 1/R) R_a/R
                const double2 cbase = make_double2(-inv * rr * base.x + rr * base.y, -inv * rr * base.y - rr * base.x);
                double acq = 1.0;
#pragma unroll
                for (int q = 0; q < kTerms; ++q) {
                    acc[j][0][q].x += acq * cbase.x;
                    acc[j][0][q].y += acq * cbase.y;
                    acc[j][1][q].x += acq * base.x;
                    acc[j][1][q].y += acq * base.y;
                    acq *= ac;
                }
                abp *= ab;
            }
        }
    }
    if (!live) return;
    double2* __restrict__ dst = Qbar + (int64_t)blockIdx.y * 2 * kTerms * kTerms * ncell;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        const int p = p0 + j;
        if (p >= kTerms) break;
        for (int f = 0; f < 2; ++f)
            for (int q = 0; q < kTerms; ++q) dst[(((int64_t)f * kTerms + p) * kTerms + q) * ncell + cell] = acc[j][f][q];
    }
}

// out = conj(x) * scale as complex64
__global__ void conj_scale_kernel(const double2* __restrict__ x, int64_t n, double scale, float2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_float2((float)(x[i].x * scale), (float)(-x[i].y * scale));
}

// Q[p][q][m][l] (GEMM output) -> [cell][field][p][q]
__global__ void reorder_q_kernel(const double2* __restrict__ Qg, int fld, int64_t ncell, double2* __restrict__ Q) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ncell * kTerms * kTerms) return;
    const int64_t cell = id % ncell;
    const int pq = (int)(id / ncell);
    Q[(cell * 2 + fld) * kTerms * kTerms + pq] = Qg[(int64_t)pq * ncell + cell];
}

// sinc(x - alpha) = sum_p s_p(x) alpha^p, s_p = (-1)^p sinc^(p)(x)/p!
void sinc_taylor(double x, double* s) {
    for (int p = 0; p <= kOrder; ++p) {
        double acc = 0.0;
        for (int j = 0; j < 40; ++j) {
            if (2 * j < p) continue;
            // (-1)^j (2j)! / ((2j-p)! (2j+1)!) x^(2j-p)
            double c = (j & 1) ? -1.0 : 1.0;
            for (int t = 2 * j - p + 1; t <= 2 * j; ++t) c *= t;
            for (int t = 2; t <= 2 * j + 1; ++t) c /= t;
            acc += c * std::pow(x, 2 * j - p);
        }
        double fact = 1.0;
        for (int t = 2; t <= p; ++t) fact *= t;
        s[p] = ((p & 1) ? -1.0 : 1.0) * acc / fact;
    }
}

}  // namespace

struct ProjectState {
    double2* phasors = nullptr;   // [face][2][plane]
    double2* spectra = nullptr;   // [face][2][plane]
    double2* work = nullptr;      // scratch
    size_t work_bytes = 0;
    double2* part = nullptr;      // per-split partial sums of the point kernels
    size_t part_bytes = 0;
    // sinc-Taylor expansion tables of the cell sums, built once per solver
    // (they depend on the grid and the box only): per face, U_p^T and V_q for
    // the points, and their conjugates in the adjoint's layout
    double2* fwd_tab = nullptr;
    double2* adj_tab = nullptr;
    int64_t fwd_off[7] = {0, 0, 0, 0, 0, 0, 0};
    int64_t adj_off[7] = {0, 0, 0, 0, 0, 0, 0};
    double2* tw = nullptr;        // per axis: twiddles exp(-2 pi i j / N)
    double2* twc = nullptr;       // per axis: conjugate twiddles
    int64_t face_off[7] = {0, 0, 0, 0, 0, 0, 0};
    int64_t total = 0;
};

namespace {

template <class T>
hipError_t ensure(T** ptr, size_t* have, size_t need) {
    if (*have >= need) return hipSuccess;
    if (*ptr) {
        (void)hipDeviceSynchronize();  // queued launches may still use the old buffer
        (void)hipFree(*ptr);
    }
    *ptr = nullptr;
    *have = 0;
    hipError_t e = hipMalloc((void**)ptr, need);
    if (e == hipSuccess) *have = need;
    return e;
}

// Rows of workgroups a point kernel is split into: enough for about eight
// waves per SIMD (256 CUs x 4 SIMDs) when the points alone give fewer, at
// most `cap` (the number of independent pieces of the summed range)
constexpr int64_t kTargetWaves = 8 * 1024;
int split_count(int64_t waves, int64_t cap) {
    int64_t k = (kTargetWaves + waves - 1) / std::max<int64_t>(waves, 1);
    k = std::min<int64_t>(k, std::min<int64_t>(cap, 64));
    return (int)std::max<int64_t>(k, 1);
}

#define TRY(x)                                \
    do {                                      \
        hipError_t _e = (x);                  \
        if (_e != hipSuccess) return _e;      \
    } while (0)

hipError_t prepare(ProjectState** pst, const pstd_problem& p, double2* const acc[3], const int64_t points[3],
                   PhasorScale scale, hipStream_t stream) {
    if (!*pst) {
        ProjectState* s = new ProjectState();
        int64_t off = 0;
        for (int f = 0; f < 6; ++f) {
            s->face_off[f] = off;
            off += 2 * points[f / 2];
        }
        s->face_off[6] = off;
        s->total = off;
        hipError_t e;
        if ((e = hipMalloc(&s->phasors, off * sizeof(double2))) || (e = hipMalloc(&s->spectra, off * sizeof(double2))) ||
            (e = hipMalloc(&s->tw, (size_t)(p.n[0] + p.n[1] + p.n[2]) * sizeof(double2))) ||
            (e = hipMalloc(&s->twc, (size_t)(p.n[0] + p.n[1] + p.n[2]) * sizeof(double2)))) {
            project_free(s);
            return e;
        }
        std::vector<double2> tw;
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < p.n[a]; ++j)
                tw.push_back(make_double2(std::cos(2 * kPi * j / p.n[a]), -std::sin(2 * kPi * j / p.n[a])));
        std::vector<double2> twc(tw);
        for (auto& v : twc) v.y = -v.y;
        if ((e = hipMemcpy(s->tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(s->twc, twc.data(), twc.size() * sizeof(double2), hipMemcpyHostToDevice))) {
            project_free(s);
            return e;
        }
        *pst = s;
    }
    ProjectState* s = *pst;
    TRY(finalize_phasors(acc, points, scale, s->phasors, stream));
    // 2D spectra of every plane
    size_t need = 0;
    for (int f = 0; f < 6; ++f) need = std::max(need, (size_t)points[f / 2] * sizeof(double2));
    TRY(ensure(&s->work, &s->work_bytes, need));
    const double2* twa[3] = {s->tw, s->tw + p.n[0], s->tw + p.n[0] + p.n[1]};
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2, b = face_axis_b(a), c = face_axis_c(a);
        const int Nb = p.n[b], Nc = p.n[c];
        const int64_t np = (int64_t)Nb * Nc;
        for (int fld = 0; fld < 2; ++fld) {
            const double2* x = s->phasors + s->face_off[f] + fld * np;
            double2* z = s->spectra + s->face_off[f] + fld * np;
            const unsigned blocks = (unsigned)((np + 255) / 256);
            hipLaunchKernelGGL(dft_rows_kernel, dim3(blocks), dim3(256), 0, stream, x, s->work, Nb, Nc, twa[b]);
            hipLaunchKernelGGL(dft_cols_kernel, dim3(blocks), dim3(256), 0, stream, s->work, z, Nb, Nc, twa[c]);
        }
    }
    return hipGetLastError();
}

}  // namespace

hipError_t finalize_phasors(double2* const acc[3], const int64_t points[3], PhasorScale scale, double2* out,
                            hipStream_t stream) {
    int64_t off = 0;
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2;
        const int64_t P = points[a];
        hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, acc[a], f % 2, P,
                           scale.v, scale.d, out + off);
        off += 2 * P;
    }
    return hipGetLastError();
}

namespace {

// Expansion of the cell integral along one face axis (axis ax, `cells` cells
// from grid index lo, FFT length N): for spectral index m (signed m') and
// cell l, the Taylor coefficients t = 0..kOrder of the sinc factor times the
// phase of the cell centre, conjugated when `conj`: put(t, l, m, value).
template <class Put>
void expansion(const double dxb[3], int ax, int lo, int cells, int N, bool conj, Put put) {
    const double d = dxb[ax], Lp = N * d;
    double sp[kTerms];
    for (int m = 0; m < N; ++m) {
        const int bp = m < N / 2 ? m : m - N;
        sinc_taylor(kPi * bp / N, sp);
        for (int l = 0; l < cells; ++l) {
            const double xc = (lo + l - N / 2 + 0.5) * d;
            const double ph = 2 * kPi * bp * xc / Lp;
            const double sg = (bp & 1) ? -1.0 : 1.0;
            const double cs = std::cos(ph), sn = conj ? -std::sin(ph) : std::sin(ph);
            for (int t = 0; t < kTerms; ++t) put(t, l, m, make_double2(sg * sp[t] * cs, sg * sp[t] * sn));
        }
    }
}

// The tables of all six faces in one device array, built on first use:
// forward (adjoint = false): U_p^T[p][b'][l] then V_q[q][m][c'];
// adjoint: Vh[c'][q][m] = conj V_q[m][c'] then Uc[p][l][b'] = conj U_p[l][b'].
hipError_t near_tables(ProjectState* s, const pstd_problem& p, const double dxb[3], bool adjoint) {
    double2*& tab = adjoint ? s->adj_tab : s->fwd_tab;
    int64_t* off = adjoint ? s->adj_off : s->fwd_off;
    if (tab) return hipSuccess;
    int64_t total = 0;
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2, b = face_axis_b(a), c = face_axis_c(a);
        const int L = p.surf_hi[b] - p.surf_lo[b], M = p.surf_hi[c] - p.surf_lo[c];
        off[f] = total;
        total += (int64_t)kTerms * (p.n[b] * L + M * p.n[c]);
    }
    off[6] = total;
    std::vector<double2> h((size_t)total);
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2, b = face_axis_b(a), c = face_axis_c(a);
        const int Nb = p.n[b], Nc = p.n[c];
        const int L = p.surf_hi[b] - p.surf_lo[b], M = p.surf_hi[c] - p.surf_lo[c];
        double2* t0 = h.data() + off[f];
        double2* t1 = t0 + (size_t)kTerms * Nb * L;
        if (!adjoint) {
            expansion(dxb, b, p.surf_lo[b], L, Nb, false,
                      [&](int t, int l, int m, double2 v) { t0[((size_t)t * Nb + m) * L + l] = v; });
            expansion(dxb, c, p.surf_lo[c], M, Nc, false,
                      [&](int t, int l, int m, double2 v) { t1[((size_t)t * M + l) * Nc + m] = v; });
        } else {
            // Vh first (Nc x kTerms M), then Uc (kTerms L x Nb): the same total
            double2* vh = t0;
            double2* uc = t0 + (size_t)Nc * kTerms * M;
            expansion(dxb, c, p.surf_lo[c], M, Nc, true,
                      [&](int t, int l, int m, double2 v) { vh[((size_t)m * kTerms + t) * M + l] = v; });
            expansion(dxb, b, p.surf_lo[b], L, Nb, true,
                      [&](int t, int l, int m, double2 v) { uc[((size_t)t * L + l) * Nb + m] = v; });
        }
    }
    hipError_t e = hipMalloc(&tab, (size_t)total * sizeof(double2));
    if (e == hipSuccess) e = hipMemcpy(tab, h.data(), (size_t)total * sizeof(double2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(tab);
        tab = nullptr;
    }
    return e;
}

}  // namespace

hipError_t far_field(ProjectState** pst, const pstd_problem& p, const double dxb[3], double2* const acc[3],
                     const int64_t points[3], PhasorScale scale, const double3* dirs, int64_t n_dir, double2* out,
                     hipStream_t stream, std::string* msg) {
    TRY(prepare(pst, p, acc, points, scale, stream));
    ProjectState* s = *pst;
    TRY(hipMemsetAsync(out, 0, n_dir * sizeof(double2), stream));
    const int64_t chunk = 8192;
    {
        // the largest scratch any face needs, allocated before the first
        // launch that uses it
        size_t need = 0;
        for (int f = 0; f < 6; ++f) {
            const int a = f / 2, Nb = p.n[face_axis_b(a)], Nc = p.n[face_axis_c(a)];
            const size_t nd = (size_t)std::min(chunk, n_dir);
            need = std::max(need, (nd * Nb + nd * Nc + (size_t)Nb * 2 * Nc + nd * 2 * Nc) * sizeof(double2));
        }
        TRY(ensure(&s->work, &s->work_bytes, need));
    }
    for (int64_t d0 = 0; d0 < n_dir; d0 += chunk) {
        const int64_t nd = std::min(chunk, n_dir - d0);
        for (int f = 0; f < 6; ++f) {
            const int a = f / 2, side = f % 2, b = face_axis_b(a), c = face_axis_c(a);
            const int Nb = p.n[b], Nc = p.n[c];
            const int idx = side == 0 ? p.surf_lo[a] : p.surf_hi[a];
            const double xa = (idx - p.n[a] / 2) * dxb[a];
            const double pref = (side == 0 ? 1.0 : -1.0) * dxb[b] * dxb[c] / (4 * kPi * Nb * Nc) / p.k0;
            // scratch: Gb [nd][Nb], Gc [nd][Nc], Mt [Nb][2Nc], T [nd][2Nc]
            double2* Gb = s->work;
            double2* Gc = Gb + nd * Nb;
            double2* Mt = Gc + nd * Nc;
            double2* T = Mt + (int64_t)Nb * 2 * Nc;
            const double2* Fp = s->spectra + s->face_off[f];
            const double2* Fd = Fp + (int64_t)Nb * Nc;
            hipLaunchKernelGGL(farfield_factor_kernel, dim3((unsigned)((nd * Nb + 255) / 256)), dim3(256), 0, stream,
                               dirs + d0, nd, b, Nb, dxb[b], p.surf_lo[b], p.surf_hi[b], Gb);
            hipLaunchKernelGGL(farfield_factor_kernel, dim3((unsigned)((nd * Nc + 255) / 256)), dim3(256), 0, stream,
                               dirs + d0, nd, c, Nc, dxb[c], p.surf_lo[c], p.surf_hi[c], Gc);
            hipLaunchKernelGGL(stack_transpose_kernel, dim3((unsigned)(((int64_t)Nb * 2 * Nc + 255) / 256)), dim3(256),
                               0, stream, Fp, Fd, Nb, Nc, Mt);
            TRY(zgemm((int)nd, 2 * Nc, Nb, Gb, Nb, 0, Mt, 2 * Nc, 0, T, 2 * Nc, 0, 1, stream));
            hipLaunchKernelGGL(farfield_dot_kernel, dim3((unsigned)((nd + kDotWaves - 1) / kDotWaves)),
                               dim3(64 * kDotWaves), 0, stream, dirs + d0, nd, a, xa, pref, Gc, T, Nc, out + d0);
        }
    }
    return hipGetLastError();
}

hipError_t project_points(ProjectState** pst, const pstd_problem& p, const double dxb[3], double2* const acc[3],
                          const int64_t points[3], PhasorScale scale, const double3* obs, int64_t n_obs, double2* out,
                          hipStream_t stream, std::string* msg) {
    // the cell formula holds outside the box only
    {
        std::vector<double3> h(n_obs);
        TRY(hipMemcpyAsync(h.data(), obs, n_obs * sizeof(double3), hipMemcpyDeviceToHost, stream));
        TRY(hipStreamSynchronize(stream));
        for (int64_t i = 0; i < n_obs; ++i) {
            const double r[3] = {h[i].x * p.k0, h[i].y * p.k0, h[i].z * p.k0};
            bool inside = true;
            for (int a = 0; a < 3; ++a) {
                const double lo = (p.surf_lo[a] - p.n[a] / 2) * dxb[a], hi = (p.surf_hi[a] - p.n[a] / 2) * dxb[a];
                if (!(r[a] > lo && r[a] < hi)) inside = false;
                if (!std::isfinite(r[a])) inside = true;
            }
            if (inside) {
                *msg = "observation point inside the box or not finite";
                return hipErrorInvalidValue;
            }
        }
    }
    TRY(prepare(pst, p, acc, points, scale, stream));
    ProjectState* s = *pst;
    TRY(near_tables(s, p, dxb, false));
    TRY(hipMemsetAsync(out, 0, n_obs * sizeof(double2), stream));
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2, side = f % 2, b = face_axis_b(a), c = face_axis_c(a);
        const int Nb = p.n[b], Nc = p.n[c];
        const int L = p.surf_hi[b] - p.surf_lo[b], M = p.surf_hi[c] - p.surf_lo[c];
        const int64_t ncell = (int64_t)L * M;
        // expansion tables U_p^T[b'][l] (batched over p) and V_q[m][c'] (batched over q)
        const double2* dUt = s->fwd_tab + s->fwd_off[f];
        const double2* dV = dUt + (size_t)kTerms * Nb * L;
        // scratch: W [p][Nc][L], Qg [p][q][M][L], Q [cell][2][p][q]
        const size_t nW = (size_t)kTerms * Nc * L, nQg = (size_t)kTerms * kTerms * ncell,
                     nQ = (size_t)2 * kTerms * kTerms * ncell;
        TRY(ensure(&s->work, &s->work_bytes, (nW + nQg + nQ) * sizeof(double2)));
        double2* dW = s->work;
        double2* dQg = dW + nW;
        double2* dQ = dQg + nQg;
        for (int fld = 0; fld < 2; ++fld) {
            const double2* F = s->spectra + s->face_off[f] + (int64_t)fld * Nb * Nc;
            // W_p = F [Nc x Nb] * Ut_p [Nb x L]
            TRY(zgemm(Nc, L, Nb, F, Nb, 0, dUt, L, (int64_t)Nb * L, dW, L, (int64_t)Nc * L, kTerms, stream));
            // Q_pq = V_q [M x Nc] * W_p [Nc x L]
            for (int pp = 0; pp < kTerms; ++pp)
                TRY(zgemm(M, L, Nc, dV, Nc, (int64_t)M * Nc, dW + (size_t)pp * Nc * L, L, 0,
                          dQg + (size_t)pp * kTerms * ncell, L, ncell, kTerms, stream));
            const int64_t tot = ncell * kTerms * kTerms;
            hipLaunchKernelGGL(reorder_q_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream, dQg, fld,
                               ncell, dQ);
        }
        FaceGeo g;
        g.a = a;
        g.b = b;
        g.c = c;
        g.lo_b = p.surf_lo[b];
        g.lo_c = p.surf_lo[c];
        g.L = L;
        g.M = M;
        g.db = dxb[b];
        g.dc = dxb[c];
        g.xa = ((side == 0 ? p.surf_lo[a] : p.surf_hi[a]) - p.n[a] / 2) * dxb[a];
        g.xb0 = (p.surf_lo[b] - Nb / 2 + 0.5) * dxb[b];
        g.xc0 = (p.surf_lo[c] - Nc / 2 + 0.5) * dxb[c];
        g.pref = (side == 0 ? 1.0 : -1.0) * dxb[b] * dxb[c] / (4 * kPi * Nb * Nc);
        const int64_t bx = (n_obs + kNearThreads * kNearPoints - 1) / (kNearThreads * kNearPoints);
        const int splits = split_count(bx * (kNearThreads / 64), (ncell + kCellChunk - 1) / kCellChunk);
        const int64_t per = (ncell + splits - 1) / splits;
        TRY(ensure(&s->part, &s->part_bytes, (size_t)splits * n_obs * sizeof(double2)));
        hipLaunchKernelGGL(near_kernel<kNearPoints>, dim3((unsigned)bx, (unsigned)splits), dim3(kNearThreads), 0, stream,
                           obs, n_obs, p.k0, g, dQ, per, s->part);
        hipLaunchKernelGGL(add_splits_kernel, dim3((unsigned)((n_obs + 255) / 256)), dim3(256), 0, stream, s->part, splits,
                           n_obs, true, out);
        // the next face reuses the scratch after these kernels, in stream order
    }
    return hipGetLastError();
}

hipError_t project_adjoint(ProjectState** pst, const pstd_problem& p, const double dxb[3], double2* const acc[3],
                           const int64_t points[3], double scale, const double3* obs, int64_t n_obs, const double2* g,
                           float2* inj, hipStream_t stream, std::string* msg) {
    // the state (twiddles, offsets) is shared with the forward projection
    TRY(prepare(pst, p, acc, points, real_scale(1.0), stream));
    ProjectState* s = *pst;
    TRY(near_tables(s, p, dxb, true));
    const double2* twc[3] = {s->twc, s->twc + p.n[0], s->twc + p.n[0] + p.n[1]};
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2, side = f % 2, b = face_axis_b(a), c = face_axis_c(a);
        const int Nb = p.n[b], Nc = p.n[c];
        const int L = p.surf_hi[b] - p.surf_lo[b], M = p.surf_hi[c] - p.surf_lo[c];
        const int64_t ncell = (int64_t)L * M, np_ = (int64_t)Nb * Nc;
        // conjugated expansion tables: Vh[c'][q M + m] = conj V_q[m][c'], Uc[p L + l][b'] = conj U_p[l][b']
        const double2* dVh = s->adj_tab + s->adj_off[f];
        const double2* dUc = dVh + (size_t)Nc * kTerms * M;
        const size_t nQ = (size_t)2 * kTerms * kTerms * ncell, nW = (size_t)Nc * kTerms * L, nF = (size_t)np_;
        TRY(ensure(&s->work, &s->work_bytes, (nQ + nW + 2 * nF) * sizeof(double2)));
        double2* dQ = s->work;
        double2* dW = dQ + nQ;
        double2* dF = dW + nW;
        double2* dT = dF + nF;
        FaceGeo geo;
        geo.a = a;
        geo.b = b;
        geo.c = c;
        geo.lo_b = p.surf_lo[b];
        geo.lo_c = p.surf_lo[c];
        geo.L = L;
        geo.M = M;
        geo.db = dxb[b];
        geo.dc = dxb[c];
        geo.xa = ((side == 0 ? p.surf_lo[a] : p.surf_hi[a]) - p.n[a] / 2) * dxb[a];
        geo.xb0 = (p.surf_lo[b] - Nb / 2 + 0.5) * dxb[b];
        geo.xc0 = (p.surf_lo[c] - Nc / 2 + 0.5) * dxb[c];
        geo.pref = (side == 0 ? 1.0 : -1.0) * dxb[b] * dxb[c] / (4 * kPi * Nb * Nc);
        const int64_t nthr = ncell * ((kTerms + kAdjP - 1) / kAdjP);
        const int64_t bx = (nthr + 127) / 128;
        const int splits = split_count(bx * 2, std::min<int64_t>((n_obs + kAdjObsChunk - 1) / kAdjObsChunk, 16));
        const int64_t per = (n_obs + splits - 1) / splits;
        const int64_t nq = 2 * kTerms * kTerms * ncell;
        double2* qdst = dQ;
        if (splits > 1) {
            TRY(ensure(&s->part, &s->part_bytes, (size_t)splits * nq * sizeof(double2)));
            qdst = s->part;
        }
        hipLaunchKernelGGL(near_adjoint_kernel<kAdjP>, dim3((unsigned)bx, (unsigned)splits), dim3(128), 0, stream, obs, g,
                           n_obs, p.k0, geo, per, qdst);
        if (splits > 1)
            hipLaunchKernelGGL(add_splits_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, stream, s->part,
                               splits, nq, false, dQ);
        for (int fld = 0; fld < 2; ++fld) {
            // Wbar[c'][p L + l] = sum_q Vh_q [Nc x M] Qbar[fld][p][q] [M x L]
            TRY(zgemm(Nc, L, kTerms * M, dVh, (int64_t)kTerms * M, 0, dQ + (size_t)fld * kTerms * kTerms * ncell, L,
                      (int64_t)kTerms * ncell, dW, (int64_t)kTerms * L, L, kTerms, stream));
            // Fbar = Wbar [Nc x 9L] * Uc [9L x Nb]
            TRY(zgemm(Nc, Nb, kTerms * L, dW, (int64_t)kTerms * L, 0, dUc, Nb, 0, dF, Nb, 0, 1, stream));
            // plane adjoint of the forward 2D DFT: the unnormalised conjugate DFT
            const unsigned blocks = (unsigned)((np_ + 255) / 256);
            hipLaunchKernelGGL(dft_rows_kernel, dim3(blocks), dim3(256), 0, stream, dF, dT, Nb, Nc, twc[b]);
            hipLaunchKernelGGL(dft_cols_kernel, dim3(blocks), dim3(256), 0, stream, dT, dF, Nb, Nc, twc[c]);
            hipLaunchKernelGGL(conj_scale_kernel, dim3(blocks), dim3(256), 0, stream, dF, np_, scale,
                               inj + s->face_off[f] + fld * np_);
        }
        // the next face reuses the scratch after these kernels, in stream order
    }
    return hipGetLastError();
}

void project_free(ProjectState* s) {
    if (!s) return;
    (void)hipFree(s->phasors);
    (void)hipFree(s->spectra);
    (void)hipFree(s->work);
    (void)hipFree(s->part);
    (void)hipFree(s->fwd_tab);
    (void)hipFree(s->adj_tab);
    (void)hipFree(s->tw);
    (void)hipFree(s->twc);
    delete s;
}

}  // namespace pstd
