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


__device__ inline v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// the plane kernel's LDS: plane [R][P] (later T), then the x and y operands
__host__ __device__ inline int dense_xy_pitch(int nx) { return 16 * ((nx + 15) / 16) + 1; }
__host__ __device__ inline int dense_xy_rows(int ny) { return 16 * ((ny + 15) / 16); }
__host__ __device__ inline int dense_frag_size(int n) { return ((n + 15) / 16) * ((n + 3) / 4) * 64; }

// One workgroup per (z plane, component, batch member): Y = B_y X B_x^T with
// X the plane less the point sources on it, for planes of up to T = 5 tiles
// of 16 per axis (KB = 4-wide k steps: the largest component's count; a
// smaller component adds zero rows and columns).  The 16 x 16 output tiles
// are dealt so that each wave needs only two tiles of the factor, which it
// keeps in registers for the whole product:
//   T = X B_x^T: wave w owns output column tile w (every row tile) and, with
//       T = 5, row tile w of column tile 4 (wave 0 also row tile 4);
//   Y = B_y T:   wave w owns output row tile w (every column tile) and, with
//       T = 5, column tile w of row tile 4 (wave 0 also column tile 4).
// Per k step a wave reads one LDS operand per row (column) tile plus one,
// and no factor from LDS.  T = X B_x^T overwrites X in LDS.
template <int KB>
__global__ void __launch_bounds__(256) dense_xy_kernel(const DenseArgs A) {
    constexpr int T = (KB + 3) / 4;
    constexpr int SH = T == 5 ? 1 : 0;  // the fifth tile row / column, shared by the waves
    static_assert(T <= 5, "planes of at most 80 x 80");
    constexpr int R = 16 * T, P = 16 * T + 1;  // plane rows and (odd) pitch in LDS
    extern __shared__ double X[];
    const int c = blockIdx.y, b = blockIdx.z, iz = blockIdx.x;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    if (iz >= nz) return;
    // the wave index as a scalar, so that the per-tile tests below are uniform branches
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int tyn = (ny + 15) / 16, txn = (nx + 15) / 16, kbx = (nx + 3) / 4, kby = (ny + 3) / 4;
    // factor tiles of this wave (indices clamped inside the factor; their
    // products with the zero padding add nothing)
    const int own_x = wv < txn ? wv : txn - 1, own_y = wv < tyn ? wv : tyn - 1;
    const double* Fx = A.frag + A.frag_off[c][0];
    const double* Fy = A.frag + A.frag_off[c][1];
    double bx[1 + SH][KB], by[1 + SH][KB];
    {
        // the plane (zero padded to R rows and P columns; rows over the waves)
        // and the factor tiles, all loads in flight together
        const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
        constexpr int RB = R / 4;
        double r0[RB], r1[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int y = wv + 4 * k;
            r0[k] = (y < ny && lane < nx) ? in[y * nx + lane] : 0.0;
            r1[k] = (y < ny && lane + 64 < nx) ? in[y * nx + lane + 64] : 0.0;
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int kx = kb < kbx ? kb : kbx - 1, ky = kb < kby ? kb : kby - 1;
            bx[0][kb] = Fx[(own_x * kbx + kx) * 64 + lane];
            by[0][kb] = Fy[(own_y * kby + ky) * 64 + lane];
            if (SH) {
                bx[SH][kb] = Fx[((txn - 1) * kbx + kx) * 64 + lane];
                by[SH][kb] = Fy[((tyn - 1) * kby + ky) * 64 + lane];
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int y = wv + 4 * k;
            if (lane < P) X[y * P + lane] = r0[k];
            if (lane + 64 < P) X[y * P + lane + 64] = r1[k];
        }
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
    // validity of the shared tiles for this component (a smaller component
    // may have fewer than five)
    const bool sh_x = SH && txn == T, sh_y = SH && tyn == T;
    v4d acc[T], acs, ace;  // own tiles, the shared tile, wave 0's corner tile
    // ---- T = X B_x^T: T[y][i] = sum_x X[y][x] B_x[i][x] ----
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    acs = ace = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        double xa[T];
#pragma unroll
        for (int t = 0; t < T; ++t) xa[t] = X[(16 * t + lr) * P + 4 * kb + lk];
        const double xw = X[(16 * wv + lr) * P + 4 * kb + lk];
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = mfma64(xa[t], bx[0][kb], acc[t]);
        if (SH) {
            acs = mfma64(xw, bx[SH][kb], acs);
            if (wv == 0) ace = mfma64(xa[T - 1], bx[SH][kb], ace);
        }
    }
    __syncthreads();  // every wave is done with X
    if (wv < txn) {
#pragma unroll
        for (int t = 0; t < T; ++t)
            if (t < tyn) {
#pragma unroll
                for (int r = 0; r < 4; ++r) X[(16 * t + lk + 4 * r) * P + 16 * wv + lr] = acc[t][r];
            }
    }
    if (SH && sh_x && wv < tyn) {
#pragma unroll
        for (int r = 0; r < 4; ++r) X[(16 * wv + lk + 4 * r) * P + 16 * (T - 1) + lr] = acs[r];
    }
    if (SH && sh_x && sh_y && wv == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) X[(16 * (T - 1) + lk + 4 * r) * P + 16 * (T - 1) + lr] = ace[r];
    }
    __syncthreads();
    // ---- Y = B_y T: Y[o][i] = sum_y B_y[o][y] T[y][i] (rows of T past ny are zero) ----
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    acs = ace = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        double ta[T];
#pragma unroll
        for (int t = 0; t < T; ++t) ta[t] = X[(4 * kb + lk) * P + 16 * t + lr];
        const double tw = X[(4 * kb + lk) * P + 16 * wv + lr];
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = mfma64(by[0][kb], ta[t], acc[t]);
        if (SH) {
            acs = mfma64(by[SH][kb], tw, acs);
            if (wv == 0) ace = mfma64(by[SH][kb], ta[T - 1], ace);
        }
    }
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
    if (wv < tyn) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int i = 16 * t + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 16 * wv + lk + 4 * r;
                if (t < txn && o < ny && i < nx) out[o * nx + i] = acc[t][r];
            }
        }
    }
    if (SH && sh_y && wv < txn) {
        const int i = 16 * wv + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 16 * (T - 1) + lk + 4 * r;
            if (o < ny && i < nx) out[o * nx + i] = acs[r];
        }
    }
    if (SH && sh_x && sh_y && wv == 0) {
        const int i = 16 * (T - 1) + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 16 * (T - 1) + lk + 4 * r;
            if (o < ny && i < nx) out[o * nx + i] = ace[r];
        }
    }
}

// One workgroup per 64 (x, y) columns of a component: out = (accumulate ? out
// : 0) + alpha B_z X over the columns, KB k steps (the largest component's;
// rows past a component's nz are zero).  Wave w owns the 16 columns 16 w ..
// 16 w + 15 and every 16-row tile of the output.  The B_z tiles (the left
// operands, the same for every wave) and the columns are read once per
// workgroup into LDS, together with the accumulated output; a k step then
// reads TZ + 1 operands from LDS for TZ products.
template <int KB>
__global__ void __launch_bounds__(256) dense_z_kernel(const DenseArgs A) {
    constexpr int TZ = (KB + 3) / 4;
    constexpr int P = 65;
    constexpr int NF = TZ * KB * 64;           // factor operands
    constexpr int LF = (NF + 255) / 256;       // factor loads per thread
    extern __shared__ double X[];  // [4 KB][P] columns, then [TZ][KB][64] factor operands
    double* F = X + 4 * KB * P;
    const int c = blockIdx.y, b = blockIdx.z;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    const int64_t ncol = int64_t(nx) * ny;
    const int64_t col0 = int64_t(blockIdx.x) * 64;
    if (col0 >= ncol) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int tzn = (nz + 15) / 16, kbz = (nz + 3) / 4;
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c];
    const int64_t col = col0 + 16 * wv + lr;
    const double* Fz = A.frag + A.frag_off[c][2];
    double o[TZ][4], fr[LF];
    {
        // the accumulated output, the factor operands and the columns (rows z
        // over the waves), all loads in flight together
#pragma unroll
        for (int t = 0; t < TZ; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int z = 16 * t + lk + 4 * r;
                o[t][r] = (A.accumulate && col < ncol && z < nz) ? out[int64_t(z) * ncol + col] : 0.0;
            }
#pragma unroll
        for (int q = 0; q < LF; ++q) {
            // operand (t, kb, l) of the padded factor; indices clamped inside the
            // stored factor (its products with the zero rows of X add nothing)
            const int i = tid + 256 * q;
            const int t = i / (KB * 64), kb = (i / 64) % KB, l = i % 64;
            const int tc = t < tzn ? t : tzn - 1, kc = kb < kbz ? kb : kbz - 1;
            const double v = Fz[i < NF ? (tc * kbz + kc) * 64 + l : 0];
            fr[q] = i < NF ? v : 0.0;
        }
        const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c];
        const bool ok = col0 + lane < ncol;
        double r[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int z = wv + 4 * k;
            r[k] = (ok && z < nz) ? in[int64_t(z) * ncol + col0 + lane] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < LF; ++q) {
            const int i = tid + 256 * q;
            if (i < NF) F[i] = fr[q];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) X[(wv + 4 * k) * P + lane] = r[k];
    }
    __syncthreads();
    v4d acc[TZ];
#pragma unroll
    for (int t = 0; t < TZ; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const double xb = X[(4 * kb + lk) * P + 16 * wv + lr];
#pragma unroll
        for (int t = 0; t < TZ; ++t) acc[t] = mfma64(F[(t * KB + kb) * 64 + lane], xb, acc[t]);
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

// k steps and plane LDS of the plane kernel for a field's components
int xy_kb(const int dims[3][3]) {
    int kb = 0;
    for (int c = 0; c < 3; ++c)
        for (int a = 1; a <= 2; ++a) {
            const int k = (dims[c][a] + 3) / 4;
            kb = k > kb ? k : kb;
        }
    return kb;
}

size_t xy_lds(const int dims[3][3]) {
    const int t = (xy_kb(dims) + 3) / 4;
    return size_t(16 * t) * (16 * t + 1) * sizeof(double);
}

int z_kb(const int dims[3][3]) {
    int kb = 0;
    for (int c = 0; c < 3; ++c) {
        const int k = (dims[c][0] + 3) / 4;
        kb = k > kb ? k : kb;
    }
    return kb;
}

size_t z_lds(const int dims[3][3]) {
    const int kb = z_kb(dims), tz = (kb + 3) / 4;
    return (size_t(4 * kb) * 65 + size_t(tz) * kb * 64) * sizeof(double);
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

template <int KB>
hipError_t raise_xy(size_t shm) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&dense_xy_kernel<KB>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
}

#define DENSE_KB_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)

template <int KB>
hipError_t raise_z(size_t shm) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&dense_z_kernel<KB>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
}

// The kernels' LDS grant only ever grows: spaces created later with smaller
// planes must not shrink what an earlier space's launches need.
hipError_t dense_prepare(size_t shm) {
    static size_t granted = 0;
    if (shm <= granted) return hipSuccess;
    hipError_t e = hipSuccess;
#define RAISE(K) \
    if (e == hipSuccess) e = raise_xy<K>(shm); \
    if (e == hipSuccess) e = raise_z<K>(shm);
    DENSE_KB_CASES(RAISE)
#undef RAISE
    if (e == hipSuccess) granted = shm;
    return e;
}

void launch_dense_xy(const DenseArgs& a, int batch, hipStream_t s) {
    int nzmax = 0;
    for (int c = 0; c < 3; ++c) nzmax = a.dims[c][0] > nzmax ? a.dims[c][0] : nzmax;
    const dim3 grid(nzmax, 3, batch);
    const size_t shm = xy_lds(a.dims);
    switch (xy_kb(a.dims)) {
#define LAUNCH(K) \
    case K: hipLaunchKernelGGL(dense_xy_kernel<K>, grid, dim3(256), shm, s, a); break;
        DENSE_KB_CASES(LAUNCH)
#undef LAUNCH
        default: break;
    }
}

void launch_dense_z(const DenseArgs& a, int batch, hipStream_t s) {
    int64_t cmax = 0;
    for (int c = 0; c < 3; ++c) {
        const int64_t n = int64_t(a.dims[c][1]) * a.dims[c][2];
        cmax = n > cmax ? n : cmax;
    }
    const dim3 grid(unsigned((cmax + 63) / 64), 3, batch);
    const size_t shm = z_lds(a.dims);
    switch (z_kb(a.dims)) {
#define LAUNCH(K) \
    case K: hipLaunchKernelGGL(dense_z_kernel<K>, grid, dim3(256), shm, s, a); break;
        DENSE_KB_CASES(LAUNCH)
#undef LAUNCH
        default: break;
    }
}

}  // namespace kmx
