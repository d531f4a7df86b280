// Tile-shape table of the pencil passes (the kernels are in pass_kernel.hpp,
// instantiated in the pass_inst<k>.hip units), and the small kernels of the
// step: FP64 norm, gradient folding, step-counter advance.
#include "pass_kernel.hpp"
#include "pass_variants.hpp"

namespace pstd {

PSTD_VARIANTS(PSTD_DECLARE_SHAPE)

namespace {

struct VariantEntry {
    PassShape shape;
    LaunchFn plain;
    LaunchFn seg;  // null when the shape has no segmented instance
    AdjFn adj;
};

const VariantEntry kVariants[] = {
#define PSTD_ENTRY(N_, A_, B_, M_, P_, S_, PART_)                                                              \
    {PassShape{N_, A_, B_, P_, P_ * (A_ > B_ ? A_ : B_), M_}, &PSTD_FN(plain, N_, A_, B_, M_, P_),                  \
     (S_) ? &PSTD_FN(seg, N_, A_, B_, M_, P_) : nullptr, &PSTD_FN(adj, N_, A_, B_, M_, P_)},
    PSTD_VARIANTS(PSTD_ENTRY)
#undef PSTD_ENTRY
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int pass_variants(int N, bool segmented, int* out, int cap) {
    int k = 0;
    for (int i = 0; i < kNumVariants; ++i) {
        if (kVariants[i].shape.N != N) continue;
        if (segmented && !kVariants[i].seg) continue;
        if (k < cap) out[k] = i;
        ++k;
    }
    return k;
}

PassShape variant_shape(int v) { return kVariants[v].shape; }

int variant_tiles(int v, int axis, PassArgs& a) {
    const int P = kVariants[v].shape.P;
    const int nseg = a.nseg > 0 ? a.nseg : 1;
    if (axis == 0) {
        a.ntx = 1;
        a.tiles = (int)(((int64_t)a.ny * a.nz * nseg + P - 1) / P);
    } else {
        a.ntx = (a.nx + P - 1) / P;
        a.tiles = a.ntx * (axis == 1 ? a.nz : a.ny) * nseg;
    }
    return a.tiles;
}

hipError_t launch_variant(int v, bool segmented, int axis, const PassArgs* descs, const int* off, int ninst,
                          int total_tiles, int koff, int potx, int nt, hipStream_t stream) {
    if (v < 0 || v >= kNumVariants || ninst < 1) return hipErrorInvalidValue;
    LaunchFn f = segmented ? kVariants[v].seg : kVariants[v].plain;
    if (!f) return hipErrorInvalidValue;
    PassArgs none{};
    none.potx = potx;   // only these fields of the by-value argument are read in a group launch
    none.nt = nt;
    return f(axis, none, descs, off, ninst, total_tiles, koff, stream);
}

hipError_t launch_variant_single(int v, bool segmented, int axis, const PassArgs& args, int koff, hipStream_t stream) {
    if (v < 0 || v >= kNumVariants) return hipErrorInvalidValue;
    LaunchFn f = segmented ? kVariants[v].seg : kVariants[v].plain;
    if (!f) return hipErrorInvalidValue;
    return f(axis, args, nullptr, nullptr, 0, args.tiles, koff, stream);
}

hipError_t launch_variant_adjoint(int v, int axis, const PassArgs& args, int koff, hipStream_t stream) {
    if (v < 0 || v >= kNumVariants) return hipErrorInvalidValue;
    return kVariants[v].adj(axis, args, koff, stream);
}

// sum |psi|^2 in FP64: per-workgroup partial sums, then one workgroup adds
// them (no atomics; a NaN or Inf anywhere makes the sum non-finite)
constexpr int kNormThreads = 256;
constexpr int kNormBlocks = 1024;

__global__ __launch_bounds__(kNormThreads) void norm_partial_kernel(const float2* __restrict__ psi, int64_t n,
                                                                    double* __restrict__ part) {
    __shared__ double red[kNormThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNormThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNormThreads) {
        const float2 v = psi[i];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kNormThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kNormThreads) void norm_final_kernel(const double* __restrict__ part, int n,
                                                                  double* __restrict__ out) {
    __shared__ double red[kNormThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kNormThreads) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kNormThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

int norm_scratch_doubles() { return kNormBlocks + 1; }

hipError_t launch_norm(const float2* psi, int64_t n, double* scratch, hipStream_t stream) {
    const int blocks = (int)std::min<int64_t>(kNormBlocks, (n + kNormThreads - 1) / kNormThreads);
    hipLaunchKernelGGL(norm_partial_kernel, dim3(blocks), dim3(kNormThreads), 0, stream, psi, n, scratch + 1);
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kNormThreads), 0, stream, scratch + 1, blocks, scratch);
    return hipGetLastError();
}

__global__ void fold_kernel(double* __restrict__ acc64, float* __restrict__ acc32, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        acc64[i] += (double)acc32[i];
        acc32[i] = 0.f;
    }
}

hipError_t launch_fold(double* acc64, float* acc32, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(fold_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, acc64, acc32, n);
    return hipGetLastError();
}

__global__ void scale_out_kernel(const double* __restrict__ acc64, double scale, float* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)(scale * acc64[i]);
}

hipError_t launch_scale_out(const double* acc64, double scale, float* out, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL(scale_out_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, acc64, scale, out, n);
    return hipGetLastError();
}

// one lane per instance: vector loads and stores of the counters
__global__ void advance_kernel(int64_t* __restrict__ ctr, int count, int by) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const int64_t n = ctr[2 * i], end = ctr[2 * i + 1];
        ctr[2 * i] = n + by < end ? n + by : (n < end ? end : n);
    }
}

hipError_t launch_advance(int64_t* ctr, int count, int by, hipStream_t stream) {
    hipLaunchKernelGGL(advance_kernel, dim3((count + 63) / 64), dim3(64), 0, stream, ctr, count, by);
    return hipGetLastError();
}

}  // namespace pstd
