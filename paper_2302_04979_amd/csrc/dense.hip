// Dense FP64 pairing solves (the tiled-dense plan).  Block c of K1 or K~1 is
// A_z (x) A_y (x) A_x (eqs. (4.2)-(4.5)), so with the inverses B_a = A_a^{-1}
// of the 1D factors formed once on the host, x = K^{-1} y is
//     X_plane <- B_y Y_plane B_x^T   for every z plane,  then  B_z along z,
// three small dense products per line instead of a serial banded
// substitution.  Both kernels run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// of the 16x4 and 4x16 operands, and register r of lane l receives
// D[l / 16 + 4 r][l % 16].
//
// The inverses are stored in operand order, frag[t][kb][lane] =
// B[16 t + lane % 16][4 kb + lane / 16] (zero outside the matrix), so that a
// wave reads one operand as 64 consecutive doubles, and the same array serves
// as the right operand of X B_x^T and the left operand of B_y T and B_z X.
#include "kernels.hpp"

namespace kmx {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int DMAX_T = DENSE_NMAX / 16;  // output tiles per axis

__device__ inline v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// the plane kernel's LDS: plane [R][P] (later T), then the x and y operands
__host__ __device__ inline int dense_xy_pitch(int nx) { return 16 * ((nx + 15) / 16) + 1; }
__host__ __device__ inline int dense_xy_rows(int ny) { return 16 * ((ny + 15) / 16); }
__host__ __device__ inline int dense_frag_size(int n) { return ((n + 15) / 16) * ((n + 3) / 4) * 64; }

// Staging global -> LDS in one round: the loads of every slot (up to S per
// thread) are issued before the first store, so a workgroup pays one memory
// latency for all of its operands.
constexpr int FRAG_SLOTS = (DMAX_T * (DENSE_NMAX / 4) * 64 + 255) / 256;  // one factor, per thread

template <int S>
struct Staged {
    double r[S];
    __device__ inline void load(const double* __restrict__ src, int n, int tid) {
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int i = u * 256 + tid;
            r[u] = i < n ? src[i] : 0.0;
        }
    }
    __device__ inline void store(double* dst, int n, int tid) const {
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int i = u * 256 + tid;
            if (i < n) dst[i] = r[u];
        }
    }
};

// One workgroup per (z plane, component, batch member): Y = B_y X B_x^T with
// X the plane less the point sources on it.  Output tiles (16 x 16) are dealt
// to the four waves, NJ per wave (the largest component's count); a wave's
// tiles past its component's count repeat its last tile and are not stored,
// so the products run without branches and the accumulators stay in the
// matrix registers.  T = X B_x^T overwrites X in LDS.
template <int NJ>
__global__ void __launch_bounds__(256) dense_xy_kernel(const DenseArgs A) {
    extern __shared__ double smem[];
    const int c = blockIdx.y, b = blockIdx.z, iz = blockIdx.x;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    if (iz >= nz) return;
    // the wave index as a scalar, so that the per-tile tests below are uniform branches
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int tyn = (ny + 15) / 16, txn = (nx + 15) / 16, kbx = (nx + 3) / 4, kby = (ny + 3) / 4;
    const int P = dense_xy_pitch(nx), R = dense_xy_rows(ny);
    double* X = smem;
    double* Fx = X + R * P;
    double* Fy = Fx + dense_frag_size(nx);
    {
        // the plane (zero padded to R rows and P columns; rows over the waves)
        // and both factors, all loads in flight together
        const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
        constexpr int RB = DENSE_NMAX / 4;
        double r0[RB], r1[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int y = wv + 4 * k;
            r0[k] = (y < ny && lane < nx) ? in[y * nx + lane] : 0.0;
            r1[k] = (y < ny && lane + 64 < nx) ? in[y * nx + lane + 64] : 0.0;
        }
        Staged<FRAG_SLOTS> fx, fy;
        fx.load(A.frag + A.frag_off[c][0], dense_frag_size(nx), tid);
        fy.load(A.frag + A.frag_off[c][1], dense_frag_size(ny), tid);
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int y = wv + 4 * k;
            if (y < R) {
                if (lane < P) X[y * P + lane] = r0[k];
                if (lane + 64 < P) X[y * P + lane + 64] = r1[k];
            }
        }
        fx.store(Fx, dense_frag_size(nx), tid);
        fy.store(Fy, dense_frag_size(ny), tid);
    }
    __syncthreads();
    if (A.n_src > 0) {
        // point sources: subtract g(t) s on this plane, in a fixed order
        if (tid == 0) {
            for (int k = A.src_off[b]; k < A.src_off[b + 1]; ++k) {
                const double* pr = A.src_prof + 4 * k;
                const double dtt = (A.t_dev ? *A.t_dev : 0.0) + A.t_src - pr[0];
                const double gt = pr[2] * exp(-dtt * dtt / (2.0 * pr[1] * pr[1]));
                const double* en = A.src_entries + int64_t(k) * A.entries_per * 5;
                for (int e = 0; e < A.entries_per; ++e) {
                    if (int(en[5 * e]) != c || int(en[5 * e + 1]) != iz) continue;
                    X[int(en[5 * e + 2]) * P + int(en[5 * e + 3])] -= gt * en[5 * e + 4];
                }
            }
        }
        __syncthreads();
    }
    const int items = tyn * txn;
    int tr[NJ], tc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        int it = wv + 4 * j;
        it = it < items ? it : (items - 1 - ((items - 1 - wv) & 3));  // this wave's last tile
        tr[j] = it / txn;
        tc[j] = it - tr[j] * txn;
    }
    v4d acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
    // T = X B_x^T: T[y][i] = sum_x X[y][x] B_x[i][x]
    for (int kb = 0; kb < kbx; ++kb) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            acc[j] = mfma64(X[(16 * tr[j] + lr) * P + 4 * kb + lk], Fx[(tc[j] * kbx + kb) * 64 + lane], acc[j]);
    }
    __syncthreads();  // every wave is done with X
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        // a repeated tile stores the same values again: harmless
#pragma unroll
        for (int r = 0; r < 4; ++r) X[(16 * tr[j] + lk + 4 * r) * P + 16 * tc[j] + lr] = acc[j][r];
        acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    __syncthreads();
    // Y = B_y T: Y[o][i] = sum_y B_y[o][y] T[y][i]  (rows of T past ny are zero)
    for (int kb = 0; kb < kby; ++kb) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            acc[j] = mfma64(Fy[(tr[j] * kby + kb) * 64 + lane], X[(4 * kb + lk) * P + 16 * tc[j] + lr], acc[j]);
    }
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (wv + 4 * j >= items) continue;
        const int i = 16 * tc[j] + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 16 * tr[j] + lk + 4 * r;
            if (o < ny && i < nx) out[o * nx + i] = acc[j][r];
        }
    }
}

// One workgroup per 64 (x, y) columns of a component: out = (accumulate ? out
// : 0) + alpha B_z X over the columns.  Wave w owns the 16 columns 16 w ..
// 16 w + 15 and the TZ 16-row tiles of the output (the largest component's
// count; a component with fewer repeats its last tile without storing it), so
// each operand of X it reads serves all of its tiles.
template <int TZ>
__global__ void __launch_bounds__(256) dense_z_kernel(const DenseArgs A) {
    extern __shared__ double smem[];
    const int c = blockIdx.y, b = blockIdx.z;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    const int64_t ncol = int64_t(nx) * ny;
    const int64_t col0 = int64_t(blockIdx.x) * 64;
    if (col0 >= ncol) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int tzn = (nz + 15) / 16, kbz = (nz + 3) / 4;
    constexpr int P = 65;
    double* X = smem;                 // [4 kbz][P]
    double* Fz = X + 4 * kbz * P;
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c];
    const int64_t col = col0 + 16 * wv + lr;
    // the accumulated output is requested first: it is not needed until the end
    double o[TZ][4];
#pragma unroll
    for (int t = 0; t < TZ; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int z = 16 * t + lk + 4 * r;
            o[t][r] = (A.accumulate && col < ncol && z < nz) ? out[int64_t(z) * ncol + col] : 0.0;
        }
    {
        // the columns (rows z over the waves) and the factor, all loads in flight together
        const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c];
        const bool ok = col0 + lane < ncol;
        constexpr int RB = DENSE_NMAX / 4;
        double r[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int z = wv + 4 * k;
            r[k] = (ok && z < nz) ? in[int64_t(z) * ncol + col0 + lane] : 0.0;
        }
        Staged<FRAG_SLOTS> fz;
        fz.load(A.frag + A.frag_off[c][2], dense_frag_size(nz), tid);
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int z = wv + 4 * k;
            if (z < 4 * kbz) X[z * P + lane] = r[k];
        }
        fz.store(Fz, dense_frag_size(nz), tid);
    }
    __syncthreads();
    v4d acc[TZ];
    int tt[TZ];
#pragma unroll
    for (int t = 0; t < TZ; ++t) {
        acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
        tt[t] = t < tzn ? t : tzn - 1;
    }
    for (int kb = 0; kb < kbz; ++kb) {
        const double xb = X[(4 * kb + lk) * P + 16 * wv + lr];
#pragma unroll
        for (int t = 0; t < TZ; ++t) acc[t] = mfma64(Fz[(tt[t] * kbz + kb) * 64 + lane], xb, acc[t]);
    }
    if (col >= ncol) return;
    const double alpha = A.alpha;
#pragma unroll
    for (int t = 0; t < TZ; ++t) {
        if (t >= tzn) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int z = 16 * t + lk + 4 * r;
            if (z < nz) out[int64_t(z) * ncol + col] = o[t][r] + alpha * acc[t][r];
        }
    }
}

size_t xy_lds(const int dims[3][3]) {
    size_t m = 0;
    for (int c = 0; c < 3; ++c) {
        const int ny = dims[c][1], nx = dims[c][2];
        const size_t s = size_t(dense_xy_rows(ny)) * dense_xy_pitch(nx) + dense_frag_size(nx) + dense_frag_size(ny);
        m = s > m ? s : m;
    }
    return m * sizeof(double);
}

size_t z_lds(const int dims[3][3]) {
    size_t m = 0;
    for (int c = 0; c < 3; ++c) {
        const int nz = dims[c][0];
        const size_t s = size_t(4 * ((nz + 3) / 4)) * 65 + dense_frag_size(nz);
        m = s > m ? s : m;
    }
    return m * sizeof(double);
}

}  // namespace

int64_t dense_frag_doubles(int n) { return dense_frag_size(n); }

void dense_fragments(const double* Bmat, int n, double* frag) {
    const int tn = (n + 15) / 16, kb = (n + 3) / 4;
    for (int t = 0; t < tn; ++t)
        for (int k = 0; k < kb; ++k)
            for (int l = 0; l < 64; ++l) {
                const int i = 16 * t + (l & 15), j = 4 * k + (l >> 4);
                frag[(size_t(t) * kb + k) * 64 + l] = (i < n && j < n) ? Bmat[size_t(i) * n + j] : 0.0;
            }
}

size_t dense_lds_bytes(const int dims[3][3]) {
    const size_t a = xy_lds(dims), b = z_lds(dims);
    return a > b ? a : b;
}

template <int NJ>
hipError_t raise_xy(size_t shm) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&dense_xy_kernel<NJ>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
}

template <int TZ>
hipError_t raise_z(size_t shm) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&dense_z_kernel<TZ>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
}

hipError_t dense_prepare(size_t shm) {
    const hipError_t e[] = {raise_xy<1>(shm), raise_xy<2>(shm), raise_xy<3>(shm), raise_xy<4>(shm),
                            raise_xy<5>(shm), raise_xy<6>(shm), raise_xy<7>(shm), raise_z<1>(shm),
                            raise_z<2>(shm),  raise_z<3>(shm),  raise_z<4>(shm),  raise_z<5>(shm)};
    for (hipError_t x : e)
        if (x != hipSuccess) return x;
    return hipSuccess;
}

void launch_dense_xy(const DenseArgs& a, int batch, hipStream_t s) {
    int nzmax = 0, items = 0;
    for (int c = 0; c < 3; ++c) {
        nzmax = a.dims[c][0] > nzmax ? a.dims[c][0] : nzmax;
        const int it = ((a.dims[c][1] + 15) / 16) * ((a.dims[c][2] + 15) / 16);
        items = it > items ? it : items;
    }
    const dim3 grid(nzmax, 3, batch);
    const size_t shm = xy_lds(a.dims);
    switch ((items + 3) / 4) {
        case 1: hipLaunchKernelGGL(dense_xy_kernel<1>, grid, dim3(256), shm, s, a); break;
        case 2: hipLaunchKernelGGL(dense_xy_kernel<2>, grid, dim3(256), shm, s, a); break;
        case 3: hipLaunchKernelGGL(dense_xy_kernel<3>, grid, dim3(256), shm, s, a); break;
        case 4: hipLaunchKernelGGL(dense_xy_kernel<4>, grid, dim3(256), shm, s, a); break;
        case 5: hipLaunchKernelGGL(dense_xy_kernel<5>, grid, dim3(256), shm, s, a); break;
        case 6: hipLaunchKernelGGL(dense_xy_kernel<6>, grid, dim3(256), shm, s, a); break;
        default: hipLaunchKernelGGL(dense_xy_kernel<7>, grid, dim3(256), shm, s, a); break;
    }
}

void launch_dense_z(const DenseArgs& a, int batch, hipStream_t s) {
    int64_t cmax = 0;
    int tz = 0;
    for (int c = 0; c < 3; ++c) {
        const int64_t n = int64_t(a.dims[c][1]) * a.dims[c][2];
        cmax = n > cmax ? n : cmax;
        const int t = (a.dims[c][0] + 15) / 16;
        tz = t > tz ? t : tz;
    }
    const dim3 grid(unsigned((cmax + 63) / 64), 3, batch);
    const size_t shm = z_lds(a.dims);
    switch (tz) {
        case 1: hipLaunchKernelGGL(dense_z_kernel<1>, grid, dim3(256), shm, s, a); break;
        case 2: hipLaunchKernelGGL(dense_z_kernel<2>, grid, dim3(256), shm, s, a); break;
        case 3: hipLaunchKernelGGL(dense_z_kernel<3>, grid, dim3(256), shm, s, a); break;
        case 4: hipLaunchKernelGGL(dense_z_kernel<4>, grid, dim3(256), shm, s, a); break;
        default: hipLaunchKernelGGL(dense_z_kernel<5>, grid, dim3(256), shm, s, a); break;
    }
}

}  // namespace kmx
