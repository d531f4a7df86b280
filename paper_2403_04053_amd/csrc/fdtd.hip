// FDTD variant of the step (Section 2.2.1; its bound Section 2.3.1): the eighth-order central stencil of
// Eq. y_stencil (coefficients of Eq. stencil_alpha) along every axis, the
// central-difference update of Eq. FDTDupdatePsi with the potential, the
// wall consistency terms of Eqs. FDTDpsi_extraJminus1-FDTDpsiJplus4 and the
// mask of Eq. expmask, in one kernel per step.
//
// The wall terms of a cell c sum, over the axes a and the stencil offsets
// l, alpha_l [T(c) - T(c +- l e_a)] psi_inc(c +- l e_a), T = 1 on the
// total-field box.  With the separable incident wave this is
// sum_a D_a(i_a) prod_{b != a} Z_b(i_b) times the step's time factor, with
// the 1D tables Z_b = T_b e^{i kh_b x_b} and D_a = -C_a e^{i kh_a x_a} /
// dxb_a^2, C_a(i) = sum_l alpha_l sum_pm [T_a(i) - T_a(i pm l)]
// e^{pm i kh_a l dxb_a}: the same form as the taper source of the spectral
// scheme, so the same per-axis tables carry it.
//
// A workgroup owns a 32 x 8 tile of (x, y) columns and a run of 16 z planes.
// Each thread keeps the nine values psi(z-4 .. z+4) of its column in VGPRs
// (the z stencil) and the plane z of the tile with a 4-cell halo is staged
// in LDS (the x and y stencils).  The loads of plane z + 1 (the halo cells,
// the next column value, psi^{n-1} and V) are issued right after plane z is
// staged, so they are in flight while plane z is computed.
// The grid is periodic (indices wrap), like the spectral passes.
#include "dft.hpp"
#include "internal.hpp"

namespace pstd {

namespace {

constexpr int kFX = 32;   // tile x (one wave row)
constexpr int kFY = 8;    // tile y
constexpr int kFH = 4;    // stencil reach
constexpr int kFZ = 16;   // z planes per workgroup
constexpr int kSX = kFX + 2 * kFH;
constexpr int kSY = kFY + 2 * kFH;

__device__ __forceinline__ int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

typedef float float2_vec __attribute__((ext_vector_type(2)));

// Five waves per SIMD: the prefetched plane needs about 96 VGPRs, and the
// register cap of six or more waves serialises its loads or spills.  NTL:
// psi^{n-1}, read here for the last time, comes in with non-temporal loads
// (chosen for fields beyond the Infinity Cache, which then keeps the
// psi^{n+1} this step writes for the next).
template <bool NTL>
__global__ __launch_bounds__(kFX * kFY) __attribute__((amdgpu_waves_per_eu(5))) void fdtd_kernel(FdtdArgs a, int koff) {
    __shared__ float2 s[kSY][kSX + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int t = ty * kFX + tx;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t nstep = a.ctr[0] + koff;
    if (nstep >= a.ctr[1]) return;  // whole workgroup, before any barrier
    const float2* __restrict__ psi = (nstep & 1) ? a.buf[1] : a.buf[0];
    float2* __restrict__ old = (nstep & 1) ? a.buf[0] : a.buf[1];
    // Workgroups are dealt round-robin to the 8 XCDs (blockIdx mod 8); give
    // each XCD a contiguous run of tiles (x fastest, then y, then z) instead,
    // so that the halo rows and planes a tile shares with its neighbours meet
    // in one L2.  A bijection of [0, G).
    const int gx = (nx + kFX - 1) / kFX, gy = (ny + kFY - 1) / kFY;
    const int G = (int)gridDim.x, gb = (int)blockIdx.x, xcd = gb & 7;
    const int gt = xcd * (G >> 3) + min(xcd, G & 7) + (gb >> 3);
    const int bx = (gt % gx) * kFX, by = ((gt / gx) % gy) * kFY;
    const int bz = gt / (gx * gy);
    const int x = bx + tx, y = by + ty;
    const bool valid = x < nx && y < ny;
    const int xw = wrap(x, nx), yw = wrap(y, ny);
    const int64_t col = xw + (int64_t)nx * yw;
    const int64_t plane = (int64_t)nx * ny;
    const int z0 = bz * kFZ;
    const int z1 = min(z0 + kFZ, nz);

    // the column psi(z0-4 .. z0+4)
    float2 q[2 * kFH + 1];
    unroll<2 * kFH + 1>([&](auto i) {
        constexpr int r = decltype(i)::value;
        q[r] = psi[col + plane * wrap(z0 - kFH + r, nz)];
    });
    // per-column factors of the mask and of the wall terms
    const float2 Zx = a.zt[0][xw], Dx = a.dz[0][xw];
    const float2 Zy = a.zt[1][yw], Dy = a.dz[1][yw];
    const float2 SA = cadd(cmul(Dx, Zy), cmul(Zx, Dy));
    const float2 SB = cmul(Zx, Zy);
    const float gxy = a.gam[0][xw] * a.gam[1][yw];
    const float2 sigma = a.sigma_tab[nstep];

    // this thread's halo cells of the staged tile (at most three: 384 halo
    // cells over 256 threads), fixed for the run: LDS slot and column offset
    constexpr int kSlots = (kSY * kSX + kFX * kFY - 1) / (kFX * kFY);
    int hslot[kSlots];
    int hcol[kSlots];  // a plane holds fewer than 2^31 cells
    unroll<kSlots>([&](auto i) {
        constexpr int j = decltype(i)::value;
        const int e = t + j * kFX * kFY;
        const int r = e / kSX, c = e % kSX;
        const bool halo = e < kSY * kSX && !(r >= kFH && r < kFH + kFY && c >= kFH && c < kFH + kFX);
        hslot[j] = halo ? e : -1;
        hcol[j] = halo ? wrap(bx + c - kFH, nx) + nx * wrap(by + r - kFH, ny) : 0;
    });
    // loads of plane z, issued one plane ahead: the halo cells and the
    // epilogue operands psi^{n-1} and V of this thread's cell
    float2 hv[kSlots];
    float2 po_n = make_float2(0.f, 0.f);
    float vv_n = 0.f;
    auto load_plane = [&](int z) {
        unroll<kSlots>([&](auto i) {
            constexpr int j = decltype(i)::value;
            if (hslot[j] >= 0) hv[j] = psi[hcol[j] + plane * z];
        });
        if (valid) {
            const int64_t ad = x + (int64_t)nx * y + plane * z;
            if constexpr (NTL) {
                const float2_vec v = __builtin_nontemporal_load((const float2_vec*)(old + ad));
                po_n = make_float2(v.x, v.y);
            } else {
                po_n = old[ad];
            }
            vv_n = a.v2[ad];
        }
    };
    if (z0 < z1) load_plane(z0);

    for (int z = z0; z < z1; ++z) {
        // stage plane z: the own column value and the prefetched halo
        s[ty + kFH][tx + kFH] = q[kFH];
        unroll<kSlots>([&](auto i) {
            constexpr int j = decltype(i)::value;
            if (hslot[j] >= 0) s[hslot[j] / kSX][hslot[j] % kSX] = hv[j];
        });
        const float2 po = po_n;
        const float vv = vv_n;
        __syncthreads();
        if (z + 1 < z1) load_plane(z + 1);  // in flight during this plane's arithmetic
        const float2 qn = psi[col + plane * wrap(z + kFH + 1, nz)];
        if (valid) {
            const float2 c0 = q[kFH];
            float2 k = cscale(c0, a.kc);
            unroll<kFH>([&](auto i) {
                constexpr int l = decltype(i)::value + 1;
                k = cadd(k, cscale(cadd(s[ty + kFH][tx + kFH - l], s[ty + kFH][tx + kFH + l]), a.k[0][l - 1]));
                k = cadd(k, cscale(cadd(s[ty + kFH - l][tx + kFH], s[ty + kFH + l][tx + kFH]), a.k[1][l - 1]));
                k = cadd(k, cscale(cadd(q[kFH - l], q[kFH + l]), a.k[2][l - 1]));
            });
            const int64_t ad = x + (int64_t)nx * y + plane * z;
            const float2 src = cadd(cmul(SA, a.zt[2][z]), cmul(SB, a.dz[2][z]));
            const float2 qq = cadd(cadd(k, cscale(c0, vv)), cmul(sigma, src));
            const float g = gxy * a.gam[2][z];
            // psi^{n+1} = Gamma (psi^{n-1} - i q)
            old[ad] = make_float2(g * (po.x + qq.y), g * (po.y - qq.x));
        }
        __syncthreads();  // the plane is read before the next one is staged
        unroll<2 * kFH>([&](auto i) {
            constexpr int r = decltype(i)::value;
            q[r] = q[r + 1];
        });
        q[2 * kFH] = qn;
    }
}

}  // namespace

const double kFdtdAlpha[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

hipError_t launch_fdtd(const FdtdArgs& a, int koff, hipStream_t stream) {
    const int tiles = ((a.nx + kFX - 1) / kFX) * ((a.ny + kFY - 1) / kFY) * ((a.nz + kFZ - 1) / kFZ);
    // psi pair and V: 20 B per cell
    const bool ntl = 20.0 * (double)a.nx * a.ny * a.nz > kInfinityCacheBytes;
    if (ntl)
        hipLaunchKernelGGL(fdtd_kernel<true>, dim3((unsigned)tiles), dim3(kFX, kFY), 0, stream, a, koff);
    else
        hipLaunchKernelGGL(fdtd_kernel<false>, dim3((unsigned)tiles), dim3(kFX, kFY), 0, stream, a, koff);
    return hipGetLastError();
}

}  // namespace pstd
