// HIP kernels (gfx950) of the scheme-2 leapfrog: fused curl + sum-factorised
// 2-form mass apply, Kronecker pairing solves one axis at a time, curls,
// pairing applies and FP64 deterministic reductions.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kmx {

// ===========================================================================
// Mass apply (Section 3.4): y_i = sum_q w^_i(q) . G(q) X(q) / gamma_e over the
// Gauss points q of every element, with X(q) the parametric vector proxy of the
// input 2-form (or of the curl of the input 1-form).  One workgroup owns a
// tile of TILE^3 elements and walks its Gauss points plane by plane in z; each
// plane is contracted with the 1D tables in three passes (z, y, x) to the
// point values, multiplied by the 3x3 metric, and contracted back (x, y, z).
// Outputs are accumulated in LDS over the tile's window of basis functions and
// written as a patch; neighbouring patches overlap and are summed, in a fixed
// order, by the solve kernel that consumes them (no atomics: bitwise
// deterministic).
// ===========================================================================
template <int P>
struct MassCfg {
    static constexpr int NQ = P + 1;
    static constexpr int Q = TILE * NQ;                   // points per tile edge
    static constexpr int NT = ((Q * Q + 63) / 64) * 64;   // one thread per point of a plane
};

template <int P, int SPACE, int C>
struct Lay {  // window layout of component C of a form space inside one tile
    static constexpr int tx = space_tag(SPACE, C, 0), ty = space_tag(SPACE, C, 1), tz = space_tag(SPACE, C, 2);
    static constexpr int Kx = tag_support(P, tx), Ky = tag_support(P, ty), Kz = tag_support(P, tz);
    static constexpr int Wx = TILE + Kx - 1, Wy = TILE + Ky - 1, Wz = TILE + Kz - 1;
    static constexpr int plane = Wx * Wy;
    static constexpr int size = plane * Wz;
};

int mass_threads(int p) {
    switch (p) {
        case 2: return MassCfg<2>::NT;
        case 3: return MassCfg<3>::NT;
        default: return MassCfg<4>::NT;
    }
}

template <int P, int SPACE>
static int64_t patch_size_t(int ntile, int64_t off[3]) {
    const int64_t nt3 = int64_t(ntile) * ntile * ntile;
    off[0] = 0;
    off[1] = nt3 * Lay<P, SPACE, 0>::size;
    off[2] = off[1] + nt3 * Lay<P, SPACE, 1>::size;
    return off[2] + nt3 * Lay<P, SPACE, 2>::size;
}

int64_t patch_size(int p, int space, int ntile, int64_t off[3]) {
#define PS(PP)                                                                          \
    if (p == PP) return space == SP_B ? patch_size_t<PP, SP_B>(ntile, off)              \
                                      : patch_size_t<PP, SP_D>(ntile, off);
    PS(2) PS(3) PS(4)
#undef PS
    return 0;
}

__device__ inline int tag_dim(int tag, int n0, int n1) { return (tag == PV || tag == DD) ? n0 : n1; }

// load one component window of a field into LDS (zero outside the space)
template <int P, class L>
__device__ inline void load_window(double* dst, const double* __restrict__ src, const int dims[3],
                                   int tx, int ty, int tz, int n0, int n1, int i) {
    const int lx = i % L::Wx, ly = (i / L::Wx) % L::Wy, lz = i / L::plane;
    const int gx = tx * TILE + tag_offset(L::tx) + lx;
    const int gy = ty * TILE + tag_offset(L::ty) + ly;
    const int gz = tz * TILE + tag_offset(L::tz) + lz;
    double v = 0.0;
    if (gx >= 0 && gx < tag_dim(L::tx, n0, n1) && gy >= 0 && gy < tag_dim(L::ty, n0, n1) && gz >= 0 &&
        gz < tag_dim(L::tz, n0, n1))
        v = src[(int64_t(gz) * dims[1] + gy) * dims[2] + gx];
    dst[i] = v;
}

// curl of the 1-form window into component C of the 2-form window:
// (d_{C+1} u_{C+2} - d_{C+2} u_{C+1}); along the differentiated axis the 1-form
// window is one entry longer, and both the primal (v[k] - v[k-1]) and the dual
// (v[r+1] - v[r]) incidence become local[l+1] - local[l].
template <int P, int SRC, int SPACE, int C>
__device__ inline double curl_at(const double* s0, const double* s1, const double* s2, int i) {
    using L = Lay<P, SPACE, C>;
    constexpr int A1 = (C + 1) % 3, A2 = (C + 2) % 3;
    using LA = Lay<P, SRC, A2>;  // differentiated along A1
    using LB = Lay<P, SRC, A1>;  // differentiated along A2
    const double* sa = (A2 == 0) ? s0 : (A2 == 1 ? s1 : s2);
    const double* sb = (A1 == 0) ? s0 : (A1 == 1 ? s1 : s2);
    const int lx = i % L::Wx, ly = (i / L::Wx) % L::Wy, lz = i / L::plane;
    int l[3] = {lx, ly, lz};
    const int ia = (l[2] * LA::Wy + l[1]) * LA::Wx + l[0];
    const int da = A1 == 0 ? 1 : (A1 == 1 ? LA::Wx : LA::plane);
    const int ib = (l[2] * LB::Wy + l[1]) * LB::Wx + l[0];
    const int db = A2 == 0 ? 1 : (A2 == 1 ? LB::Wx : LB::plane);
    return (sa[ia + da] - sa[ia]) - (sb[ib + db] - sb[ib]);
}

template <int P, class L>
__device__ inline void stage_z(const double* xin, double* zpl, const double* __restrict__ t, int lez, int i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < L::Kz; ++j) s += t[j] * xin[(lez + j) * L::plane + i];
    zpl[i] = s;
}

template <int P, class L>
__device__ inline void stage_y(const double* zpl, double* ypl, const double* __restrict__ tab, int ty, int i) {
    constexpr int NQ = P + 1;
    const int lx = i % L::Wx, qy = i / L::Wx;
    const int ley = qy / NQ, iqy = qy % NQ;
    const double* t = tab + ((ty * TILE + ley) * NQ + iqy) * L::Ky;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < L::Ky; ++j) s += t[j] * zpl[(ley + j) * L::Wx + lx];
    ypl[i] = s;
}

template <int P, class L>
__device__ inline double stage_x(const double* ypl, const double* __restrict__ tab, int tx, int qy, int qx) {
    constexpr int NQ = P + 1;
    const int lex = qx / NQ, iqx = qx % NQ;
    const double* t = tab + ((tx * TILE + lex) * NQ + iqx) * L::Kx;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < L::Kx; ++j) s += t[j] * ypl[qy * L::Wx + lex + j];
    return s;
}

template <int P, class L>
__device__ inline void stage_xt(const double* uq, double* xt, const double* __restrict__ tab, int tx, int i) {
    constexpr int NQ = P + 1, Q = TILE * NQ;
    const int lx = i % L::Wx, qy = i / L::Wx;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < L::Kx; ++j) {
        const int lex = lx - j;
        if (lex < 0 || lex >= TILE) continue;
        const double* t = tab + ((tx * TILE + lex) * NQ) * L::Kx + j;
#pragma unroll
        for (int iq = 0; iq < NQ; ++iq) s += t[iq * L::Kx] * uq[qy * Q + lex * NQ + iq];
    }
    xt[i] = s;
}

template <int P, class L>
__device__ inline void stage_yt(const double* xt, double* yt, const double* __restrict__ tab, int ty, int i) {
    constexpr int NQ = P + 1;
    const int lx = i % L::Wx, ly = i / L::Wx;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < L::Ky; ++j) {
        const int ley = ly - j;
        if (ley < 0 || ley >= TILE) continue;
        const double* t = tab + ((ty * TILE + ley) * NQ) * L::Ky + j;
#pragma unroll
        for (int iq = 0; iq < NQ; ++iq) s += t[iq * L::Ky] * xt[(ley * NQ + iq) * L::Wx + lx];
    }
    yt[i] = s;
}

template <int P, class L>
__device__ inline void stage_zt(const double* yt, double* acc, const double* __restrict__ t, int lez, int i) {
    const double v = yt[i];
#pragma unroll
    for (int j = 0; j < L::Kz; ++j) acc[(lez + j) * L::plane + i] += t[j] * v;
}

template <int P, int SPACE, bool CURL>
__global__ void __launch_bounds__(MassCfg<P>::NT) mass_kernel(const MassArgs A) {
    constexpr int NQ = P + 1, Q = TILE * NQ, NT = MassCfg<P>::NT;
    constexpr int SRC = CURL ? (SPACE == SP_B ? SP_E : SP_H) : SPACE;
    using L0 = Lay<P, SPACE, 0>;
    using L1 = Lay<P, SPACE, 1>;
    using L2 = Lay<P, SPACE, 2>;
    using S0 = Lay<P, SRC, 0>;
    using S1 = Lay<P, SRC, 1>;
    using S2 = Lay<P, SRC, 2>;
    // LDS map: input window | accumulators | 1-form window | plane scratch
    constexpr int OX0 = 0, OX1 = OX0 + L0::size, OX2 = OX1 + L1::size, OXE = OX2 + L2::size;
    constexpr int OA0 = OXE, OA1 = OA0 + L0::size, OA2 = OA1 + L1::size, OAE = OA2 + L2::size;
    constexpr int OS0 = OAE, OS1 = OS0 + (CURL ? S0::size : 0), OS2 = OS1 + (CURL ? S1::size : 0),
                  OSE = OS2 + (CURL ? S2::size : 0);
    // z-contracted plane / y-transposed plane share storage
    constexpr int OZ0 = OSE, OZ1 = OZ0 + L0::plane, OZ2 = OZ1 + L1::plane, OZE = OZ2 + L2::plane;
    // y-contracted rows / x-transposed rows share storage
    constexpr int OY0 = OZE, OY1 = OY0 + Q * L0::Wx, OY2 = OY1 + Q * L1::Wx, OYE = OY2 + Q * L2::Wx;
    constexpr int OU0 = OYE, OU1 = OU0 + Q * Q, OU2 = OU1 + Q * Q, OUE = OU2 + Q * Q;
    __shared__ double sm[OUE];

    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    const int b = blockIdx.y;
    const int nt = A.ntile;
    const int tx = tile % nt, ty = (tile / nt) % nt, tz = tile / (nt * nt);
    const double* src = A.src + int64_t(b) * A.src_stride;

    // ---- input window (with the curl fused) ----
    if (CURL) {
        for (int i = tid; i < S0::size + S1::size + S2::size; i += NT) {
            if (i < S0::size)
                load_window<P, S0>(sm + OS0, src + A.src_comp_off[0], A.src_dims[0], tx, ty, tz, A.n0, A.n1, i);
            else if (i < S0::size + S1::size)
                load_window<P, S1>(sm + OS1, src + A.src_comp_off[1], A.src_dims[1], tx, ty, tz, A.n0, A.n1,
                                   i - S0::size);
            else
                load_window<P, S2>(sm + OS2, src + A.src_comp_off[2], A.src_dims[2], tx, ty, tz, A.n0, A.n1,
                                   i - S0::size - S1::size);
        }
        __syncthreads();
        for (int i = tid; i < L0::size + L1::size + L2::size; i += NT) {
            if (i < L0::size)
                sm[OX0 + i] = curl_at<P, SRC, SPACE, 0>(sm + OS0, sm + OS1, sm + OS2, i);
            else if (i < L0::size + L1::size)
                sm[OX1 + i - L0::size] = curl_at<P, SRC, SPACE, 1>(sm + OS0, sm + OS1, sm + OS2, i - L0::size);
            else
                sm[OX2 + i - L0::size - L1::size] =
                    curl_at<P, SRC, SPACE, 2>(sm + OS0, sm + OS1, sm + OS2, i - L0::size - L1::size);
        }
    } else {
        for (int i = tid; i < L0::size + L1::size + L2::size; i += NT) {
            if (i < L0::size)
                load_window<P, L0>(sm + OX0, src + A.src_comp_off[0], A.src_dims[0], tx, ty, tz, A.n0, A.n1, i);
            else if (i < L0::size + L1::size)
                load_window<P, L1>(sm + OX1, src + A.src_comp_off[1], A.src_dims[1], tx, ty, tz, A.n0, A.n1,
                                   i - L0::size);
            else
                load_window<P, L2>(sm + OX2, src + A.src_comp_off[2], A.src_dims[2], tx, ty, tz, A.n0, A.n1,
                                   i - L0::size - L1::size);
        }
    }
    for (int i = tid; i < OAE - OA0; i += NT) sm[OA0 + i] = 0.0;
    __syncthreads();

    const double* tab0x = A.tab + A.tab_off[L0::tx];
    const double* tab0y = A.tab + A.tab_off[L0::ty];
    const double* tab0z = A.tab + A.tab_off[L0::tz];
    const double* tab1x = A.tab + A.tab_off[L1::tx];
    const double* tab1y = A.tab + A.tab_off[L1::ty];
    const double* tab1z = A.tab + A.tab_off[L1::tz];
    const double* tab2x = A.tab + A.tab_off[L2::tx];
    const double* tab2y = A.tab + A.tab_off[L2::ty];
    const double* tab2z = A.tab + A.tab_off[L2::tz];

    const int qy = tid / Q, qx = tid % Q;
    const bool active = tid < Q * Q;
    const int ex = tx * TILE + qx / NQ, ey = ty * TILE + qy / NQ;
    const double* metric_tile = A.metric + int64_t(tile) * Q * 6 * Q * Q;

    for (int qz = 0; qz < Q; ++qz) {
        const int lez = qz / NQ, iqz = qz % NQ, ez = tz * TILE + lez;
        const double* t0z = tab0z + (ez * NQ + iqz) * L0::Kz;
        const double* t1z = tab1z + (ez * NQ + iqz) * L1::Kz;
        const double* t2z = tab2z + (ez * NQ + iqz) * L2::Kz;
        // prefetch this thread's metric entries early
        double g[6] = {0, 0, 0, 0, 0, 0};
        double ig = 1.0;
        if (active) {
            const double* gm = metric_tile + int64_t(qz) * 6 * Q * Q + qy * Q + qx;
#pragma unroll
            for (int k = 0; k < 6; ++k) g[k] = gm[k * Q * Q];
            if (A.inv_gamma) ig = A.inv_gamma[(int64_t(ez) * A.npad + ey) * A.npad + ex];
        }
        // z pass
        for (int i = tid; i < L0::plane + L1::plane + L2::plane; i += NT) {
            if (i < L0::plane) stage_z<P, L0>(sm + OX0, sm + OZ0, t0z, lez, i);
            else if (i < L0::plane + L1::plane) stage_z<P, L1>(sm + OX1, sm + OZ1, t1z, lez, i - L0::plane);
            else stage_z<P, L2>(sm + OX2, sm + OZ2, t2z, lez, i - L0::plane - L1::plane);
        }
        __syncthreads();
        // y pass
        for (int i = tid; i < Q * (L0::Wx + L1::Wx + L2::Wx); i += NT) {
            if (i < Q * L0::Wx) stage_y<P, L0>(sm + OZ0, sm + OY0, tab0y, ty, i);
            else if (i < Q * (L0::Wx + L1::Wx)) stage_y<P, L1>(sm + OZ1, sm + OY1, tab1y, ty, i - Q * L0::Wx);
            else stage_y<P, L2>(sm + OZ2, sm + OY2, tab2y, ty, i - Q * (L0::Wx + L1::Wx));
        }
        __syncthreads();
        // x pass, metric, store point values
        if (active) {
            const double v0 = stage_x<P, L0>(sm + OY0, tab0x, tx, qy, qx);
            const double v1 = stage_x<P, L1>(sm + OY1, tab1x, tx, qy, qx);
            const double v2 = stage_x<P, L2>(sm + OY2, tab2x, tx, qy, qx);
            sm[OU0 + qy * Q + qx] = ig * (g[0] * v0 + g[3] * v1 + g[4] * v2);
            sm[OU1 + qy * Q + qx] = ig * (g[3] * v0 + g[1] * v1 + g[5] * v2);
            sm[OU2 + qy * Q + qx] = ig * (g[4] * v0 + g[5] * v1 + g[2] * v2);
        }
        __syncthreads();
        // x^T pass
        for (int i = tid; i < Q * (L0::Wx + L1::Wx + L2::Wx); i += NT) {
            if (i < Q * L0::Wx) stage_xt<P, L0>(sm + OU0, sm + OY0, tab0x, tx, i);
            else if (i < Q * (L0::Wx + L1::Wx)) stage_xt<P, L1>(sm + OU1, sm + OY1, tab1x, tx, i - Q * L0::Wx);
            else stage_xt<P, L2>(sm + OU2, sm + OY2, tab2x, tx, i - Q * (L0::Wx + L1::Wx));
        }
        __syncthreads();
        // y^T pass
        for (int i = tid; i < L0::plane + L1::plane + L2::plane; i += NT) {
            if (i < L0::plane) stage_yt<P, L0>(sm + OY0, sm + OZ0, tab0y, ty, i);
            else if (i < L0::plane + L1::plane) stage_yt<P, L1>(sm + OY1, sm + OZ1, tab1y, ty, i - L0::plane);
            else stage_yt<P, L2>(sm + OY2, sm + OZ2, tab2y, ty, i - L0::plane - L1::plane);
        }
        __syncthreads();
        // z^T accumulation (each (c, y, x) column owned by one thread)
        for (int i = tid; i < L0::plane + L1::plane + L2::plane; i += NT) {
            if (i < L0::plane) stage_zt<P, L0>(sm + OZ0, sm + OA0, t0z, lez, i);
            else if (i < L0::plane + L1::plane) stage_zt<P, L1>(sm + OZ1, sm + OA1, t1z, lez, i - L0::plane);
            else stage_zt<P, L2>(sm + OZ2, sm + OA2, t2z, lez, i - L0::plane - L1::plane);
        }
        __syncthreads();
    }
    // write the tile's patch
    double* out = A.patch + int64_t(b) * A.patch_stride;
    for (int i = tid; i < L0::size + L1::size + L2::size; i += NT) {
        if (i < L0::size) out[A.patch_comp_off[0] + int64_t(tile) * L0::size + i] = sm[OA0 + i];
        else if (i < L0::size + L1::size)
            out[A.patch_comp_off[1] + int64_t(tile) * L1::size + (i - L0::size)] = sm[OA0 + i];
        else
            out[A.patch_comp_off[2] + int64_t(tile) * L2::size + (i - L0::size - L1::size)] = sm[OA0 + i];
    }
}

void launch_mass(int p, int space, bool curl, const MassArgs& a, int batch, hipStream_t s) {
    const int nt3 = a.ntile * a.ntile * a.ntile;
    dim3 grid(nt3, batch);
#define LM(PP)                                                                                           \
    if (p == PP) {                                                                                       \
        if (space == SP_B) {                                                                             \
            if (curl) hipLaunchKernelGGL((mass_kernel<PP, SP_B, true>), grid, dim3(MassCfg<PP>::NT), 0, s, a);  \
            else hipLaunchKernelGGL((mass_kernel<PP, SP_B, false>), grid, dim3(MassCfg<PP>::NT), 0, s, a);      \
        } else {                                                                                         \
            if (curl) hipLaunchKernelGGL((mass_kernel<PP, SP_D, true>), grid, dim3(MassCfg<PP>::NT), 0, s, a);  \
            else hipLaunchKernelGGL((mass_kernel<PP, SP_D, false>), grid, dim3(MassCfg<PP>::NT), 0, s, a);      \
        }                                                                                                \
        return;                                                                                          \
    }
    LM(2) LM(3) LM(4)
#undef LM
}

// ===========================================================================
// Pairing solves (eqs. (4.4), (4.5)): block c of K1 or K~1 is A_z (x) A_y (x) A_x,
// so K^{-1} applies A_x^{-1}, A_y^{-1}, A_z^{-1} along the lines of each axis.
// Each 1D solve is a banded forward/backward substitution with the
// precomputed LU factors (half bandwidth W = p-1).
// ===========================================================================
template <int W>
__device__ inline void band_solve_line(double* v, int n, int stride, const double* __restrict__ L,
                                       const double* __restrict__ U, const double* __restrict__ dinv) {
    double prev[W];
#pragma unroll
    for (int k = 0; k < W; ++k) prev[k] = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = v[i * stride];
#pragma unroll
        for (int k = 0; k < W; ++k) s -= L[i * W + k] * prev[k];
#pragma unroll
        for (int k = W - 1; k > 0; --k) prev[k] = prev[k - 1];
        prev[0] = s;
        v[i * stride] = s;
    }
#pragma unroll
    for (int k = 0; k < W; ++k) prev[k] = 0.0;
    for (int i = n - 1; i >= 0; --i) {
        double s = v[i * stride];
#pragma unroll
        for (int k = 0; k < W; ++k) s -= U[i * W + k] * prev[k];
        s *= dinv[i];
#pragma unroll
        for (int k = W - 1; k > 0; --k) prev[k] = prev[k - 1];
        prev[0] = s;
        v[i * stride] = s;
    }
}

struct FacView {
    const double *L, *U, *dinv;
};
template <int W>
__device__ inline FacView fac_view(const double* fac, const int64_t* fac_off, int id, int n) {
    const double* base = fac + fac_off[id];
    return {base, base + int64_t(n) * W, base + int64_t(2) * n * W};
}

// patch window geometry along one axis for gathering
template <int P>
__device__ inline int tag_window(int tag) { return TILE + tag_support(P, tag) - 1; }

template <int P, int SPACE>
__device__ inline double gather_patch(const XYArgs& A, const double* patch, int c, int gz, int gy, int gx) {
    const int nt = A.ntile;
    int tg[3], W[3], g[3] = {gx, gy, gz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        tg[a] = space_tag(SPACE, c, a);
        W[a] = TILE + tag_support(P, tg[a]) - 1;
    }
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int r = g[a] - tag_offset(tg[a]);  // >= 0
        int t1 = r / TILE;
        if (t1 > nt - 1) t1 = nt - 1;
        int t0 = t1;
        if (t1 - 1 >= 0 && r - (t1 - 1) * TILE < W[a]) t0 = t1 - 1;
        lo[a] = t0;
        hi[a] = t1;
    }
    const double* base = patch + A.patch_comp_off[c];
    const int size = W[0] * W[1] * W[2];
    double s = 0.0;
    for (int tz = lo[2]; tz <= hi[2]; ++tz)
        for (int ty = lo[1]; ty <= hi[1]; ++ty)
            for (int tx = lo[0]; tx <= hi[0]; ++tx) {
                const int lx = g[0] - tx * TILE - tag_offset(tg[0]);
                const int ly = g[1] - ty * TILE - tag_offset(tg[1]);
                const int lz = g[2] - tz * TILE - tag_offset(tg[2]);
                if (lx < 0 || lx >= W[0] || ly < 0 || ly >= W[1] || lz < 0 || lz >= W[2]) continue;
                const int64_t tile = (int64_t(tz) * nt + ty) * nt + tx;
                s += base[tile * size + (lz * W[1] + ly) * W[0] + lx];
            }
    return s;
}

template <int P, int SPACE>
__global__ void __launch_bounds__(256) xy_kernel(const XYArgs A) {
    constexpr int W = P - 1;
    extern __shared__ double plane[];
    const int c = blockIdx.y, b = blockIdx.z, iz = blockIdx.x;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    if (iz >= nz) return;
    const int nxp = nx | 1;  // odd row stride: x-lines hit distinct LDS banks
    const int tid = threadIdx.x;
    // gather
    if (A.from_patch) {
        const double* patch = A.patch + int64_t(b) * A.patch_stride;
        for (int i = tid; i < nx * ny; i += blockDim.x) {
            const int x = i % nx, y = i / nx;
            plane[y * nxp + x] = gather_patch<P, SPACE>(A, patch, c, iz, y, x);
        }
    } else {
        const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
        for (int i = tid; i < nx * ny; i += blockDim.x) plane[(i / nx) * nxp + (i % nx)] = in[i];
    }
    __syncthreads();
    // point sources: subtract g(t) s on this plane, in a fixed order
    if (A.n_src > 0 && tid == 0) {
        for (int k = A.src_off[b]; k < A.src_off[b + 1]; ++k) {
            const double* pr = A.src_prof + 4 * k;
            const double dtt = A.t_src - pr[0];
            const double gt = pr[2] * exp(-dtt * dtt / (2.0 * pr[1] * pr[1]));
            const double* en = A.src_entries + int64_t(k) * A.entries_per * 5;
            for (int e = 0; e < A.entries_per; ++e) {
                if (int(en[5 * e]) != c || int(en[5 * e + 1]) != iz) continue;
                plane[int(en[5 * e + 2]) * nxp + int(en[5 * e + 3])] -= gt * en[5 * e + 4];
            }
        }
    }
    __syncthreads();
    if (A.solve) {
        const FacView fx = fac_view<W>(A.fac, A.fac_off, A.fac_id[c][0], nx);
        const FacView fy = fac_view<W>(A.fac, A.fac_off, A.fac_id[c][1], ny);
        for (int y = tid; y < ny; y += blockDim.x) band_solve_line<W>(plane + y * nxp, nx, 1, fx.L, fx.U, fx.dinv);
        __syncthreads();
        for (int x = tid; x < nx; x += blockDim.x) band_solve_line<W>(plane + x, ny, nxp, fy.L, fy.U, fy.dinv);
        __syncthreads();
    }
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
    for (int i = tid; i < nx * ny; i += blockDim.x) out[i] = plane[(i / nx) * nxp + (i % nx)];
}

void launch_xy(int p, const XYArgs& a, int batch, hipStream_t s) {
    int nzmax = 0, smax = 0;
    for (int c = 0; c < 3; ++c) {
        nzmax = a.dims[c][0] > nzmax ? a.dims[c][0] : nzmax;
        const int sz = a.dims[c][1] * (a.dims[c][2] | 1);
        smax = sz > smax ? sz : smax;
    }
    dim3 grid(nzmax, 3, batch);
    const size_t shm = size_t(smax) * sizeof(double);
    const int space = a.gather_space;
#define LX(PP)                                                                                         \
    if (p == PP) {                                                                                     \
        if (space == SP_D) hipLaunchKernelGGL((xy_kernel<PP, SP_D>), grid, dim3(256), shm, s, a);      \
        else hipLaunchKernelGGL((xy_kernel<PP, SP_B>), grid, dim3(256), shm, s, a);                    \
        return;                                                                                        \
    }
    LX(2) LX(3) LX(4)
#undef LX
}

// z solve: one thread per (x, y) column, 64 columns per workgroup staged in LDS.
template <int P>
__global__ void __launch_bounds__(64) z_kernel(const ZArgs A) {
    constexpr int W = P - 1;
    extern __shared__ double col[];  // [nz][64]
    const int c = blockIdx.y, b = blockIdx.z;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    const int64_t ncol = int64_t(nx) * ny;
    const int64_t colid = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (int64_t(blockIdx.x) * 64 >= ncol) return;
    const bool ok = colid < ncol;
    const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c];
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c];
    const int t = threadIdx.x;
    // stage the column block (loads batched so many are in flight)
    for (int z0 = 0; z0 < nz; z0 += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (ok && z0 + k < nz) ? in[int64_t(z0 + k) * ncol + colid] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (z0 + k < nz) col[(z0 + k) * 64 + t] = v[k];
    }
    if (A.solve) {
        const FacView fz = fac_view<W>(A.fac, A.fac_off, A.fac_id[c], nz);
        band_solve_line<W>(col + t, nz, 64, fz.L, fz.U, fz.dinv);
    }
    if (!ok) return;
    const double alpha = A.alpha;
    if (A.accumulate) {
        for (int z0 = 0; z0 < nz; z0 += 8) {
            double o[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) o[k] = (z0 + k < nz) ? out[int64_t(z0 + k) * ncol + colid] : 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (z0 + k < nz) out[int64_t(z0 + k) * ncol + colid] = o[k] + alpha * col[(z0 + k) * 64 + t];
        }
    } else {
        for (int z = 0; z < nz; ++z) out[int64_t(z) * ncol + colid] = alpha * col[z * 64 + t];
    }
}

void launch_z(int p, const ZArgs& a, int batch, hipStream_t s) {
    int64_t colmax = 0;
    int nzmax = 0;
    for (int c = 0; c < 3; ++c) {
        const int64_t n = int64_t(a.dims[c][1]) * a.dims[c][2];
        colmax = n > colmax ? n : colmax;
        nzmax = a.dims[c][0] > nzmax ? a.dims[c][0] : nzmax;
    }
    dim3 grid(unsigned((colmax + 63) / 64), 3, batch);
    const size_t shm = size_t(nzmax) * 64 * sizeof(double);
#define LZ(PP)                                                                \
    if (p == PP) {                                                            \
        hipLaunchKernelGGL((z_kernel<PP>), grid, dim3(64), shm, s, a);        \
        return;                                                               \
    }
    LZ(2) LZ(3) LZ(4)
#undef LZ
}

// ===========================================================================
// Curl (incidence matrices, Section 2.4): out = beta out + alpha (d_{c+1} u_{c+2}
// - d_{c+2} u_{c+1}); primal d: v[k] - v[k-1] (zero outside), dual d~: v[r+1] - v[r].
// ===========================================================================
__device__ inline double diff1(const double* u, const int d[3], int primal, int axis, int z, int y, int x) {
    int i[3] = {x, y, z};
    const int n = d[2 - axis];
    auto at = [&](int k) -> double {
        int j[3] = {i[0], i[1], i[2]};
        j[axis] = k;
        if (k < 0 || k >= n) return 0.0;
        return u[(int64_t(j[2]) * d[1] + j[1]) * d[2] + j[0]];
    };
    const int k = i[axis];
    return primal ? at(k) - at(k - 1) : at(k + 1) - at(k);
}

__global__ void curl_kernel(const CurlArgs A, int64_t n_out) {
    const int b = blockIdx.y;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    int c = 0;
    while (c < 2 && i >= A.out_comp_off[c + 1]) ++c;
    const int64_t li = i - A.out_comp_off[c];
    const int* od = A.out_dims[c];
    const int x = int(li % od[2]), y = int((li / od[2]) % od[1]), z = int(li / (int64_t(od[2]) * od[1]));
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    const double* in = A.in + int64_t(b) * A.in_stride;
    const double v = diff1(in + A.in_comp_off[a2], A.in_dims[a2], A.primal, a1, z, y, x) -
                     diff1(in + A.in_comp_off[a1], A.in_dims[a1], A.primal, a2, z, y, x);
    double* out = A.out + int64_t(b) * A.out_stride;
    out[i] = (A.beta == 0.0 ? 0.0 : A.beta * out[i]) + A.alpha * v;
}

void launch_curl(const CurlArgs& a, int64_t n_out, int batch, hipStream_t s) {
    dim3 grid(unsigned((n_out + 255) / 256), batch);
    hipLaunchKernelGGL(curl_kernel, grid, dim3(256), 0, s, a, n_out);
}

// ===========================================================================
// Pairing apply y = K x (banded Kronecker product, for energies and tests).
// ===========================================================================
template <int P>
__device__ inline double kron_band_at(const double* in, const int d[3], const double* bx, const double* by,
                                      const double* bz, int z, int y, int x) {
    constexpr int W = P - 1, BW = 2 * W + 1;
    double s = 0.0;
    for (int kz = 0; kz < BW; ++kz) {
        const int jz = z - W + kz;
        if (jz < 0 || jz >= d[0]) continue;
        const double az = bz[z * BW + kz];
        for (int ky = 0; ky < BW; ++ky) {
            const int jy = y - W + ky;
            if (jy < 0 || jy >= d[1]) continue;
            const double ay = az * by[y * BW + ky];
            const double* row = in + (int64_t(jz) * d[1] + jy) * d[2];
            double sx = 0.0;
            for (int kx = 0; kx < BW; ++kx) {
                const int jx = x - W + kx;
                if (jx < 0 || jx >= d[2]) continue;
                sx += bx[x * BW + kx] * row[jx];
            }
            s += ay * sx;
        }
    }
    return s;
}

template <int P>
__global__ void pairing_kernel(const PairArgs A, int64_t n) {
    constexpr int W = P - 1;
    const int b = blockIdx.y;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    while (c < 2 && i >= A.comp_off[c + 1]) ++c;
    const int64_t li = i - A.comp_off[c];
    const int* d = A.dims[c];
    const int x = int(li % d[2]), y = int((li / d[2]) % d[1]), z = int(li / (int64_t(d[2]) * d[1]));
    const double* bnd[3];
    for (int a = 0; a < 3; ++a) {
        const int nn = d[2 - a];
        bnd[a] = A.fac + A.fac_off[A.fac_id[c][a]] + int64_t(nn) * (2 * W + 1);  // band block
    }
    const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c];
    A.out[int64_t(b) * A.out_stride + i] = kron_band_at<P>(in, d, bnd[0], bnd[1], bnd[2], z, y, x);
}

void launch_pairing(int p, const PairArgs& a, int64_t n, int batch, hipStream_t s) {
    dim3 grid(unsigned((n + 255) / 256), batch);
    if (p == 2) hipLaunchKernelGGL(pairing_kernel<2>, grid, dim3(256), 0, s, a, n);
    else if (p == 3) hipLaunchKernelGGL(pairing_kernel<3>, grid, dim3(256), 0, s, a, n);
    else hipLaunchKernelGGL(pairing_kernel<4>, grid, dim3(256), 0, s, a, n);
}

// ===========================================================================
// Energies (3.2) and the leapfrog invariant, FP64, deterministic tree sums.
// term0 = d . (K1 e), term1 = b . (K~1 h), term2 = (K~1 h) . (D^1 e)
// ===========================================================================
template <int NTH>
__device__ inline void block_sum3(double v0, double v1, double v2, double* out) {
    __shared__ double s[3][NTH];
    s[0][threadIdx.x] = v0;
    s[1][threadIdx.x] = v1;
    s[2][threadIdx.x] = v2;
    __syncthreads();
    for (int h = NTH / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[k] = s[k][0];
}

template <int P>
__global__ void __launch_bounds__(256) energy_kernel(const EnergyArgs A) {
    constexpr int W = P - 1;
    const int b = blockIdx.y;
    const double* e = A.E + int64_t(b) * 2 * A.n_e;
    const double* dvec = e + A.n_e;
    const double* h = A.H + int64_t(b) * 2 * A.n_h;
    const double* bvec = h + A.n_h;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    const int64_t nmax = A.n_e > A.n_h ? A.n_e : A.n_h;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nmax; i += int64_t(gridDim.x) * 256) {
        if (i < A.n_e) {  // d-space index: (K1 e)_i d_i
            int c = 0;
            while (c < 2 && i >= A.e_comp_off[c + 1]) ++c;
            const int64_t li = i - A.e_comp_off[c];
            const int* d = A.e_dims[c];
            const int x = int(li % d[2]), y = int((li / d[2]) % d[1]), z = int(li / (int64_t(d[2]) * d[1]));
            // band block of a factor set sits after L, U (n*W each) and dinv (n)
            const double* bnd[3];
            for (int a = 0; a < 3; ++a) {
                const int nn = d[2 - a];
                bnd[a] = A.fac + A.fac_off[a == c ? F_M : F_G] + int64_t(nn) * (2 * W + 1);
            }
            const double v = kron_band_at<P>(e + A.e_comp_off[c], d, bnd[0], bnd[1], bnd[2], z, y, x);
            t0 += v * dvec[i];
        }
        if (i < A.n_h) {  // b-space index: (K~1 h)_i (b_i, (D^1 e)_i)
            int c = 0;
            while (c < 2 && i >= A.h_comp_off[c + 1]) ++c;
            const int64_t li = i - A.h_comp_off[c];
            const int* d = A.h_dims[c];
            const int x = int(li % d[2]), y = int((li / d[2]) % d[1]), z = int(li / (int64_t(d[2]) * d[1]));
            const double* bnd[3];
            for (int a = 0; a < 3; ++a) {
                const int nn = d[2 - a];
                bnd[a] = A.fac + A.fac_off[a == c ? F_GT : F_MT] + int64_t(nn) * (2 * W + 1);
            }
            const double u = kron_band_at<P>(h + A.h_comp_off[c], d, bnd[0], bnd[1], bnd[2], z, y, x);
            const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
            const double w = diff1(e + A.e_comp_off[a2], A.e_dims[a2], 1, a1, z, y, x) -
                             diff1(e + A.e_comp_off[a1], A.e_dims[a1], 1, a2, z, y, x);
            t1 += u * bvec[i];
            t2 += u * w;
        }
    }
    block_sum3<256>(t0, t1, t2, A.partial + (int64_t(b) * A.nblocks + blockIdx.x) * 3);
}

void launch_energy(int p, const EnergyArgs& a, int batch, hipStream_t s) {
    dim3 grid(a.nblocks, batch);
    if (p == 2) hipLaunchKernelGGL(energy_kernel<2>, grid, dim3(256), 0, s, a);
    else if (p == 3) hipLaunchKernelGGL(energy_kernel<3>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(energy_kernel<4>, grid, dim3(256), 0, s, a);
}

__global__ void __launch_bounds__(256) energy_final_kernel(const double* partial, int nblocks, double dt,
                                                           double* out, int64_t out_stride) {
    const int b = blockIdx.x;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += 256) {
        const double* p = partial + (int64_t(b) * nblocks + k) * 3;
        t0 += p[0];
        t1 += p[1];
        t2 += p[2];
    }
    __shared__ double r[3];
    block_sum3<256>(t0, t1, t2, r);
    if (threadIdx.x == 0) {
        const double paper = 0.5 * (r[0] + r[1]);
        out[int64_t(b) * out_stride] = paper - 0.5 * dt * r[2];
        if (out_stride >= 2) out[int64_t(b) * out_stride + 1] = paper;
    }
}

void launch_energy_final(const double* partial, int nblocks, double dt, int batch, double* out,
                         int64_t out_stride, hipStream_t s) {
    hipLaunchKernelGGL(energy_final_kernel, dim3(batch), dim3(256), 0, s, partial, nblocks, dt, out, out_stride);
}

// ===========================================================================
// Dot products and vector updates (CFL power iteration, CG).
// ===========================================================================
__global__ void __launch_bounds__(256) dot_kernel(const double* x, const double* y, int64_t n, int64_t stride,
                                                  double* partial, int nblocks) {
    const int b = blockIdx.y;
    const double* xb = x + int64_t(b) * stride;
    const double* yb = y + int64_t(b) * stride;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        s += xb[i] * yb[i];
    __shared__ double r[3];
    block_sum3<256>(s, 0.0, 0.0, r);
    if (threadIdx.x == 0) partial[int64_t(b) * nblocks + blockIdx.x] = r[0];
}

void launch_dot(const double* x, const double* y, int64_t n, int64_t stride, int batch, double* partial,
                int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(dot_kernel, dim3(nblocks, batch), dim3(256), 0, s, x, y, n, stride, partial, nblocks);
}

__global__ void __launch_bounds__(256) sum_final_kernel(const double* partial, int nblocks, double* out) {
    const int b = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += 256) s += partial[int64_t(b) * nblocks + k];
    __shared__ double r[3];
    block_sum3<256>(s, 0.0, 0.0, r);
    if (threadIdx.x == 0) out[b] = r[0];
}

void launch_sum_final(const double* partial, int nblocks, int batch, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_final_kernel, dim3(batch), dim3(256), 0, s, partial, nblocks, out);
}

__global__ void axpby_kernel(const double* x, double* y, int64_t n, double ka, const double* sa, double kb) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = sa ? sa[0] * ka : ka;
    y[i] = a * x[i] + (kb == 0.0 ? 0.0 : kb * y[i]);
}

void launch_axpby(const double* x, double* y, int64_t n, double ka, const double* sa, double kb, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, x, y, n, ka, sa, kb);
}

// Conjugate-gradient vector updates with scalars kept on the device:
// scal[0] = r.z, scal[1] = p.Ap, scal[2] = new r.z.
//   phase 0: x += a p, r -= a Ap        (a = scal[0] / scal[1])
//   phase 1: p = z + beta p             (beta = scal[2] / scal[0])
__global__ void cg_kernel(double* x, double* r, double* pdir, const double* Ap, const double* z, int64_t n,
                          const double* scal, int phase) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (phase == 0) {
        const double a = scal[0] / scal[1];
        x[i] += a * pdir[i];
        r[i] -= a * Ap[i];
    } else {
        const double beta = scal[2] / scal[0];
        pdir[i] = z[i] + beta * pdir[i];
    }
}

void launch_cg_update(double* x, double* r, double* pdir, const double* Ap, const double* z, int64_t n,
                      const double* scal, int phase, hipStream_t s) {
    hipLaunchKernelGGL(cg_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, x, r, pdir, Ap, z, n, scal,
                       phase);
}

}  // namespace kmx
