// Mixed-precision pairing solves: x = K^{-1} y with the Kronecker factors of
// K (eqs. (4.2)-(4.3)) inverted densely once on the host (FP64, rounded to
// FP32) and applied as three mode-n products in FP32 on the matrix cores
// (v_mfma_f32_16x16x4_f32, FP32 accumulation).  Accuracy is won back by
// iterative refinement with the FP64 banded residual r = y - K x computed by
// the line kernels (the FP64 1D factors never leave FP64).
//
// One mode product along `axis` of a component tensor (dims [z, y, x]) is
//     out[line][i] = sum_j A[i][j] in[line][j],   i, j < n = dims[2 - axis],
// over all lines of that axis: a GEMM with the small dense n x n factor on the
// left and the lines as columns.  A workgroup takes 64 lines: the lines and
// the factor are staged in LDS (zero padded to multiples of 16 and 4), each of
// its four waves accumulates a 16-line slice for every 16-row tile of A.
#include "kernels.hpp"

namespace kmx {

namespace {

constexpr int MODE_NMAX = 80;   // padded factor size (lines of up to 80 entries)
constexpr int MODE_LINES = 64;  // lines per workgroup
static_assert(MODE_NMAX * MODE_NMAX % 256 == 0 && MODE_NMAX * MODE_LINES % 256 == 0, "staging slots");

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline int64_t line_base(int axis, int l, int ny, int nx) {
    if (axis == 0) return int64_t(l) * nx;                               // l = z*ny + y
    if (axis == 1) return int64_t(l / nx) * ny * nx + (l % nx);          // l = z*nx + x
    return l;                                                            // l = y*nx + x
}

__global__ void __launch_bounds__(256) mode_kernel(const ModeArgs M) {
    __shared__ float As[MODE_NMAX][MODE_NMAX + 4];
    __shared__ float Xs[MODE_NMAX][MODE_LINES + 4];
    const int c = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
    const int* d = M.dims[c];
    const int ny = d[1], nx = d[2];
    const int n = d[2 - M.axis];
    const int nlines = d[0] * ny * nx / n;
    const int l0 = blockIdx.x * MODE_LINES;
    if (l0 >= nlines) return;  // uniform over the workgroup
    const int64_t sj = M.axis == 0 ? 1 : (M.axis == 1 ? nx : int64_t(ny) * nx);
    // dense factor (zero padded) and the block of lines (contiguous index
    // fastest across threads); every load of a thread is issued before the
    // first LDS store
    constexpr int NA = MODE_NMAX * MODE_NMAX / 256, NX = MODE_NMAX * MODE_LINES / 256;
    const float* A = M.A + M.A_off[c];
    const int64_t in_base = int64_t(b) * M.in_stride + M.comp_off[c];
    float ra[NA], rx[NX];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int i = tid + q * 256, r = i / MODE_NMAX, k = i % MODE_NMAX;
        ra[q] = (r < n && k < n) ? A[r * n + k] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        const int i = tid + q * 256;
        const int j = M.axis == 0 ? i % MODE_NMAX : i / MODE_LINES;
        const int l = M.axis == 0 ? i / MODE_NMAX : i % MODE_LINES;
        const int lg = l0 + l;
        rx[q] = 0.0f;
        if (j < n && lg < nlines) {
            const int64_t at = in_base + line_base(M.axis, lg, ny, nx) + j * sj;
            rx[q] = M.in_f64 ? float(static_cast<const double*>(M.in)[at]) : static_cast<const float*>(M.in)[at];
        }
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int i = tid + q * 256;
        As[i / MODE_NMAX][i % MODE_NMAX] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        const int i = tid + q * 256;
        const int j = M.axis == 0 ? i % MODE_NMAX : i / MODE_LINES;
        const int l = M.axis == 0 ? i / MODE_NMAX : i % MODE_LINES;
        Xs[j][l] = rx[q];
    }
    __syncthreads();
    const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    const int ntile = (n + 15) / 16;
    v4f acc[MODE_NMAX / 16];
#pragma unroll
    for (int t = 0; t < MODE_NMAX / 16; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < n; k0 += 4) {
        const float bv = Xs[k0 + lk][16 * w + lr];
#pragma unroll
        for (int t = 0; t < MODE_NMAX / 16; ++t) {
            if (t < ntile) {
                const float av = As[16 * t + lr][k0 + lk];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
            }
        }
    }
    // lane holds rows 16t + 4 lk + r of line 16 w + lr
    const int lg = l0 + 16 * w + lr;
    if (lg >= nlines) return;
    const int64_t out_base = int64_t(b) * M.out_stride + M.comp_off[c] + line_base(M.axis, lg, ny, nx);
#pragma unroll
    for (int t = 0; t < MODE_NMAX / 16; ++t) {
        if (t < ntile) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * t + 4 * lk + r;
                if (i < n) {
                    const int64_t at = out_base + i * sj;
                    if (M.out_kind == 0) static_cast<float*>(M.out)[at] = acc[t][r];
                    else if (M.out_kind == 1) static_cast<double*>(M.out)[at] = double(acc[t][r]);
                    else static_cast<double*>(M.out)[at] += M.alpha * double(acc[t][r]);
                }
            }
        }
    }
}

__global__ void strided_axpy_kernel(const double* __restrict__ x, int64_t xs, double* __restrict__ y, int64_t ys,
                                    int64_t n, double alpha) {
    const int b = blockIdx.y;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[b * ys + i] += alpha * x[b * xs + i];
}

}  // namespace

int mode_line_max() { return MODE_NMAX; }

void launch_mode(const ModeArgs& a, int batch, hipStream_t s) {
    int lines = 0;
    for (int c = 0; c < 3; ++c) {
        const int l = a.dims[c][0] * a.dims[c][1] * a.dims[c][2] / a.dims[c][2 - a.axis];
        lines = l > lines ? l : lines;
    }
    dim3 grid((lines + MODE_LINES - 1) / MODE_LINES, 3, batch);
    hipLaunchKernelGGL(mode_kernel, grid, dim3(256), 0, s, a);
}

void launch_strided_axpy(const double* x, int64_t xs, double* y, int64_t ys, int64_t n, double alpha, int batch,
                         hipStream_t s) {
    dim3 grid(unsigned((n + 255) / 256), batch);
    hipLaunchKernelGGL(strided_axpy_kernel, grid, dim3(256), 0, s, x, xs, y, ys, n, alpha);
}

}  // namespace kmx
