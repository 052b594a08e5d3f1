// HIP kernels (gfx950) of the scheme-2 leapfrog: fused curl + sum-factorised
// 2-form mass apply, Kronecker pairing solves one axis at a time, curls,
// pairing applies and FP64 deterministic reductions.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "patch.hpp"

namespace kmx {

// ===========================================================================
// Mass apply (Section 3.4): y_i = sum_q w^_i(q) . G(q) X(q) / gamma_e over the
// Gauss points q of every element, with X(q) the parametric vector proxy of the
// input 2-form (or of the curl of the input 1-form).  The same kernel applies
// the 1-form masses of the first scheme (Section 3.3): there G(q) is the
// covariant factor det DF (DF^T DF)^{-1} and the material multiplies,
// y_i = sum_q w^_i(q) . G(q) X(q) gamma_e; the per-element array the kernel
// reads holds 1/gamma for 2-forms and gamma for 1-forms.  One workgroup owns a
// tile of TILE^3 elements and one thread owns one (x, y) Gauss-point column
// of it.  Sum factorisation in three parts:
//   1. the tile's coefficient window is contracted along y and x once (LDS),
//      leaving each thread a register column A[cz] over the z window;
//   2. the thread walks its column's Gauss points in z without barriers: z
//      contraction from A, the 3x3 metric (streamed from HBM, the only large
//      operand), and the z integral accumulated into a register column R[cz];
//   3. the R columns are contracted back along x and y once (LDS).
// Outputs cover the tile's window of basis functions and are written as a
// patch; neighbouring patches overlap and are summed, in a fixed order, by the
// solve kernel that consumes them (no atomics: bitwise deterministic).
// ===========================================================================
// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// block index; block i is given tile (i mod 8) * (T/8) + i / 8 so that every
// XCD walks one contiguous range of tiles (whole z layers at 64^3) and the
// windows that neighbouring tiles share stay in that XCD's L2.
__device__ inline int xcd_tile(int block, int ntiles) {
    constexpr int XCD = 8;
    const int per = ntiles / XCD;
    return block < per * XCD ? (block % XCD) * per + block / XCD : block;
}

// 1/d for d in a modest range (here det DF of the analytic map, in [0.7, 1.3]):
// the hardware reciprocal estimate refined by two Newton steps
// r <- r + r (1 - d r), each squaring the relative error, so the result is
// within rounding of the IEEE quotient at a fraction of its cost.
__device__ inline double recip_nr(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

template <int P>
struct MassCfg {
    static constexpr int NQ = P + 1;
    static constexpr int Q = TILE * NQ;                   // points per tile edge
    static constexpr int NT = ((Q * Q + 63) / 64) * 64;   // one thread per point of a plane
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
    if (p == PP) return space == SP_B   ? patch_size_t<PP, SP_B>(ntile, off)            \
                      : space == SP_D   ? patch_size_t<PP, SP_D>(ntile, off)            \
                      : space == SP_E   ? patch_size_t<PP, SP_E>(ntile, off)            \
                                        : patch_size_t<PP, SP_H>(ntile, off);
    PS(2) PS(3) PS(4)
#undef PS
    return 0;
}

__device__ inline int tag_dim(int tag, int n0, int n1) { return (tag == PV || tag == DD) ? n0 : n1; }

// value of one entry of a component window of a field (zero outside the space)
template <int P, class L>
__device__ inline double window_value(const double* __restrict__ src, const int dims[3], int tx, int ty, int tz,
                                      int n0, int n1, int i) {
    const int lx = i % L::Wx, ly = (i / L::Wx) % L::Wy, lz = i / L::plane;
    const int gx = tx * TILE + tag_offset(L::tx) + lx;
    const int gy = ty * TILE + tag_offset(L::ty) + ly;
    const int gz = tz * TILE + tag_offset(L::tz) + lz;
    double v = 0.0;
    if (gx >= 0 && gx < tag_dim(L::tx, n0, n1) && gy >= 0 && gy < tag_dim(L::ty, n0, n1) && gz >= 0 &&
        gz < tag_dim(L::tz, n0, n1))
        v = src[(int64_t(gz) * dims[1] + gy) * dims[2] + gx];
    return v;
}

// the three component windows of a field into LDS (contiguous, component after
// component); every load of a thread is issued before its first LDS store
template <int P, class L0, class L1, class L2, int NT>
__device__ inline void load_windows(double* dst, const double* __restrict__ src, const int64_t comp_off[3],
                                    const int dims[3][3], int tx, int ty, int tz, int n0, int n1, int tid) {
    constexpr int TOT = L0::size + L1::size + L2::size;
    constexpr int IT = (TOT + NT - 1) / NT;
    double r[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int i = tid + k * NT;
        r[k] = 0.0;
        if (i < L0::size) r[k] = window_value<P, L0>(src + comp_off[0], dims[0], tx, ty, tz, n0, n1, i);
        else if (i < L0::size + L1::size)
            r[k] = window_value<P, L1>(src + comp_off[1], dims[1], tx, ty, tz, n0, n1, i - L0::size);
        else if (i < TOT)
            r[k] = window_value<P, L2>(src + comp_off[2], dims[2], tx, ty, tz, n0, n1, i - L0::size - L1::size);
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int i = tid + k * NT;
        if (i < TOT) dst[i] = r[k];
    }
}

// Component window rows for the mass kernel: lane (g, ly, lx) = (tid / 64,
// (tid / 8) % 8, tid % 8) holds the entries (lx, ly, g + k G) of the window
// (G = NT / 64 z-groups), so the index arithmetic and the x, y bounds tests
// are done once per thread and the eight lanes of an x row read contiguous
// memory.
template <int P, class L, int G, int I>
__device__ inline void window_rows(double (&r)[I], const double* __restrict__ src, const int dims[3], int tx, int ty,
                                   int tz, int n0, int n1, int lx, int ly, int g) {
    static_assert(L::Wx <= 8 && L::Wy <= 8, "an (x, y) plane of a window fits 64 lanes");
    const int gx = tx * TILE + tag_offset(L::tx) + lx;
    const int gy = ty * TILE + tag_offset(L::ty) + ly;
    const bool okxy = lx < L::Wx && ly < L::Wy && gx >= 0 && gx < tag_dim(L::tx, n0, n1) && gy >= 0 &&
                      gy < tag_dim(L::ty, n0, n1);
    const int nz = tag_dim(L::tz, n0, n1);
    const int gz0 = tz * TILE + tag_offset(L::tz) + g;
    const int64_t zs = int64_t(dims[1]) * dims[2];
#pragma unroll
    for (int k = 0; k < I; ++k) {
        // branch-free: the load comes from index 0 where the entry is outside
        const int lz = g + k * G, gz = gz0 + k * G;
        const bool ok = okxy && lz < L::Wz && gz >= 0 && gz < nz;
        const double t = src[ok ? int64_t(gz) * zs + int64_t(gy) * dims[2] + gx : 0];
        r[k] = ok ? t : 0.0;
    }
}

template <class L, int G, int I>
__device__ inline void store_rows(double* dst, const double (&r)[I], int lx, int ly, int g) {
#pragma unroll
    for (int k = 0; k < I; ++k) {
        const int lz = g + k * G;
        if (lx < L::Wx && ly < L::Wy && lz < L::Wz) dst[(lz * L::Wy + ly) * L::Wx + lx] = r[k];
    }
}

// curl of the 1-form window into component C of the 2-form window:
// (d_{C+1} u_{C+2} - d_{C+2} u_{C+1}); along the differentiated axis the 1-form
// window is one entry longer, and both the primal (v[k] - v[k-1]) and the dual
// (v[r+1] - v[r]) incidence become local[l+1] - local[l].
template <int P, int SRC, int SPACE, int C>
__device__ inline double curl_xyz(const double* s0, const double* s1, const double* s2, int lx, int ly, int lz) {
    constexpr int A1 = (C + 1) % 3, A2 = (C + 2) % 3;
    using LA = Lay<P, SRC, A2>;  // differentiated along A1
    using LB = Lay<P, SRC, A1>;  // differentiated along A2
    const double* sa = (A2 == 0) ? s0 : (A2 == 1 ? s1 : s2);
    const double* sb = (A1 == 0) ? s0 : (A1 == 1 ? s1 : s2);
    const int ia = (lz * LA::Wy + ly) * LA::Wx + lx;
    constexpr int da = A1 == 0 ? 1 : (A1 == 1 ? LA::Wx : LA::plane);
    const int ib = (lz * LB::Wy + ly) * LB::Wx + lx;
    constexpr int db = A2 == 0 ? 1 : (A2 == 1 ? LB::Wx : LB::plane);
    return (sa[ia + da] - sa[ia]) - (sb[ib + db] - sb[ib]);
}

// the same at entry i of the 2-form window of component C
template <int P, int SRC, int SPACE, int C>
__device__ inline double curl_at(const double* s0, const double* s1, const double* s2, int i) {
    using L = Lay<P, SPACE, C>;
    return curl_xyz<P, SRC, SPACE, C>(s0, s1, s2, i % L::Wx, (i / L::Wx) % L::Wy, i / L::plane);
}

// The tile that owns global index g of a window along one axis: the tile t with
// t * TILE <= g - offset < (t + 1) * TILE (the last tile also owns the tail).
template <int TAG>
__device__ inline int owner_tile(int g, int nt) {
    int t = (g - tag_offset(TAG)) / TILE;
    return t > nt - 1 ? nt - 1 : t;
}

// The entries of the y column (lx, ., lz) of a component window that this tile
// owns: their offsets in the tracked component (-1 where not owned) and their
// current values, requested at the start of the tile so that the update in
// the y pass does not wait for them.  Branch-free (a lane that owns nothing
// reads index 0 and keeps -1): nested early exits would make the compiler
// rebuild the two arrays' initial values at every exit.
template <class L, int NY>
__device__ inline void track_column_load(const double* __restrict__ tr, const int dims[3], int tx, int ty, int tz,
                                         int nt, int lane, int (&k)[NY], double (&v)[NY]) {
    const int lz = lane / L::Wx, lx = lane - lz * L::Wx;
    const int gx = tx * TILE + tag_offset(L::tx) + lx;
    const int gz = tz * TILE + tag_offset(L::tz) + lz;
    const bool ok = lane < L::Wz * L::Wx && gx >= 0 && gx < dims[2] && gz >= 0 && gz < dims[0] &&
                    owner_tile<L::tx>(gx, nt) == tx && owner_tile<L::tz>(gz, nt) == tz;
#pragma unroll
    for (int ly = 0; ly < NY; ++ly) {
        const int gy = ty * TILE + tag_offset(L::ty) + ly;
        const bool own = ok && ly < L::Wy && gy >= 0 && gy < dims[1] && owner_tile<L::ty>(gy, nt) == ty;
        const int off = own ? (gz * dims[1] + gy) * dims[2] + gx : 0;
        const double t = tr[off];
        k[ly] = own ? off : -1;
        v[ly] = own ? t : 0.0;
    }
}

// Table slot of axis a: 0 = the tag of the component along a, 1 = the tag of
// the two components across a.
template <int SPACE>
__device__ constexpr int slot_of(int c, int a) { return c == a ? 0 : 1; }

// Per-component register columns: A (values of the input after the x and y
// contractions, one per z-window entry) and R (z-accumulated integrals).
template <int P, class L, int NQ, int Q>
__device__ inline void contract_xy(const double* __restrict__ xw, double* bb, const double* tabx,
                                   const double* taby, double (&Acol)[L::Wz], int tid, int NT, int qy, int qx,
                                   bool active) {
    // y contraction of every z-plane of the window: bb[cz][qy][lx]
    for (int i = tid; i < L::Wz * Q * L::Wx; i += NT) {
        const int cz = i / (Q * L::Wx), r = i % (Q * L::Wx);
        const int q = r / L::Wx, lx = r % L::Wx;
        const int le = q / NQ, iq = q % NQ;
        const double* t = taby + (le * NQ + iq) * L::Ky;
        const double* x = xw + (cz * L::Wy + le) * L::Wx + lx;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < L::Ky; ++j) s += t[j] * x[j * L::Wx];
        bb[i] = s;
    }
    __syncthreads();
    // x contraction into this thread's register column
    if (active) {
        const int le = qx / NQ, iq = qx % NQ;
        double phi[L::Kx];
#pragma unroll
        for (int j = 0; j < L::Kx; ++j) phi[j] = tabx[(le * NQ + iq) * L::Kx + j];
#pragma unroll
        for (int cz = 0; cz < L::Wz; ++cz) {
            const double* b = bb + (cz * Q + qy) * L::Wx + le;
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < L::Kx; ++j) s += phi[j] * b[j];
            Acol[cz] = s;
        }
    }
    __syncthreads();
}

template <int P, class L, int NQ, int Q>
__device__ inline void integrate_xy(const double (&Rcol)[L::Wz], double* rb, double* bb, const double* tabx,
                                    const double* taby, double* __restrict__ out, int tid, int NT, int qy, int qx,
                                    bool active) {
    if (active) {
#pragma unroll
        for (int cz = 0; cz < L::Wz; ++cz) rb[(cz * Q + qy) * (Q + 1) + qx] = Rcol[cz];
    }
    __syncthreads();
    // transposed x contraction: bb[cz][qy][lx]
    for (int i = tid; i < L::Wz * Q * L::Wx; i += NT) {
        const int cz = i / (Q * L::Wx), r = i % (Q * L::Wx);
        const int q = r / L::Wx, lx = r % L::Wx;
        const double* row = rb + (cz * Q + q) * (Q + 1);  // odd pitch: rows spread over the banks
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < L::Kx; ++j) {
            const int le = lx - j;
            if (le < 0 || le >= TILE) continue;
#pragma unroll
            for (int iq = 0; iq < NQ; ++iq) s += tabx[(le * NQ + iq) * L::Kx + j] * row[le * NQ + iq];
        }
        bb[i] = s;
    }
    __syncthreads();
    // transposed y contraction straight into the tile's patch
    for (int i = tid; i < L::size; i += NT) {
        const int cz = i / L::plane, r = i % L::plane;
        const int ly = r / L::Wx, lx = r % L::Wx;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < L::Ky; ++j) {
            const int le = ly - j;
            if (le < 0 || le >= TILE) continue;
#pragma unroll
            for (int iq = 0; iq < NQ; ++iq)
                s += taby[(le * NQ + iq) * L::Ky + j] * bb[(cz * Q + le * NQ + iq) * L::Wx + lx];
        }
        out[i] = s;
    }
}

// ---- pieces of the mass kernel ---------------------------------------------
// The 1D tables are the same for every lane of a workgroup except along x.
// The y tables and the x tables of the integrals are read from global memory
// with uniform addresses (the scalar cache); the x tables of the contraction
// (indexed by lane) and the z tables (used in the register-heavy Gauss-point
// walk, where scalar registers run short) are staged in LDS.

// table of axis a and slot (0: the tag of the component along a, 1: the tag of
// the components across a) for the tile coordinate `coord` along a:
// [element][point][function]
template <int P, int SPACE, int AX, int SLOT>
__device__ inline const double* axis_table(const double* __restrict__ tab, const int64_t* tab_off, int coord) {
    constexpr int tag = SLOT == 0 ? space_tag(SPACE, AX, AX) : space_tag(SPACE, (AX + 1) % 3, AX);
    return tab + tab_off[tag] + int64_t(coord) * (TILE * (P + 1) * tag_support(P, tag));
}

// LDS pitches of one component: the y-contracted window yc[cz][qy][lx], whose
// z planes are padded so that consecutive planes start Wx entries apart modulo
// 16 doubles (the planes one wave writes then fall on distinct banks), and
// the x-integrated rows xi[cz][lx][qy] (odd row pitch), which reuse its space.
template <class L, int Q>
struct MassPitch {
    static constexpr int bz = Q * L::Wx + ((L::Wx - Q * L::Wx) % 16 + 16) % 16;
    static constexpr int yc = L::Wz * bz;
    static constexpr int xi = L::Wz * L::Wx * (Q + 1);
    static constexpr int size = yc > xi ? yc : xi;
};

// Part 1a, one wave per component: lane (cz, lx) takes the y column of the
// component's window at (lx, cz) -- formed from the 1-form windows when the
// curl is fused -- adds the entries this tile owns to the tracked 2-form, and
// contracts the column along y: yc[cz][qy][lx] = sum_j T_y[qy][j] x[le(qy) + j].
template <int P, int SRC, int SPACE, int C, bool CURL, int NQ, int Q, int NY>
__device__ inline void forward_y(const double* s0, const double* s1, const double* s2, const double* xw,
                                 double* yc, const double* __restrict__ tyt, int lane, double* __restrict__ tr,
                                 const MassArgs& A, const int (&tk)[NY], const double (&tv)[NY]) {
    using L = Lay<P, SPACE, C>;
    using PT = MassPitch<L, Q>;
    if (lane >= L::Wz * L::Wx) return;
    const int cz = lane / L::Wx, lx = lane - cz * L::Wx;
    double x[L::Wy];
#pragma unroll
    for (int ly = 0; ly < L::Wy; ++ly)
        x[ly] = CURL ? curl_xyz<P, SRC, SPACE, C>(s0, s1, s2, lx, ly, cz) : xw[(cz * L::Wy + ly) * L::Wx + lx];
    if (CURL && tr) {
        double* t = tr + A.track_comp_off[C];
#pragma unroll
        for (int ly = 0; ly < L::Wy; ++ly)
            if (tk[ly] >= 0) t[tk[ly]] = tv[ly] + A.track_alpha * x[ly];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int le = q / NQ;
        const double* t = tyt + q * L::Ky;
        double s = t[0] * x[le];
#pragma unroll
        for (int j = 1; j < L::Ky; ++j) s = fma(t[j], x[le + j], s);
        yc[cz * PT::bz + q * L::Wx + lx] = s;
    }
}

// Part 1b: thread (qy, qx) contracts along x into its register column,
// A[cz] = sum_j T_x[qx][j] yc[cz][qy][le(qx) + j].
template <class L, int NQ, int Q>
__device__ inline void forward_x(const double* yc, const double* txl, double (&Acol)[L::Wz], int qy, int qx) {
    using PT = MassPitch<L, Q>;
    const int le = qx / NQ;
    double phi[L::Kx];
#pragma unroll
    for (int j = 0; j < L::Kx; ++j) phi[j] = txl[qx * L::Kx + j];
#pragma unroll
    for (int cz = 0; cz < L::Wz; ++cz) {
        const double* b = yc + cz * PT::bz + qy * L::Wx + le;
        double s = phi[0] * b[0];
#pragma unroll
        for (int j = 1; j < L::Kx; ++j) s = fma(phi[j], b[j], s);
        Acol[cz] = s;
    }
}

// Part 3a: thread t = (cz, qy) integrates one x row of the z integrals R
// against the x table: xi[cz][lx][qy] = sum over (qx, j) with le(qx) + j = lx
// of T_x[qx][j] R[cz][qy][qx].
template <class L, int NQ, int Q>
__device__ inline void integrate_x_row(const double* rb, double* xi, const double* __restrict__ txt, int t) {
    if (t >= L::Wz * Q) return;
    const int cz = t / Q, qy = t - cz * Q;
    const double* row = rb + t * (Q + 1);
    double r[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) r[k] = row[k];
    double c[L::Wx];
#pragma unroll
    for (int lx = 0; lx < L::Wx; ++lx) c[lx] = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int le = q / NQ;
#pragma unroll
        for (int j = 0; j < L::Kx; ++j) c[le + j] = fma(txt[q * L::Kx + j], r[q], c[le + j]);
    }
#pragma unroll
    for (int lx = 0; lx < L::Wx; ++lx) xi[(cz * L::Wx + lx) * (Q + 1) + qy] = c[lx];
}

// Part 3b, one wave per component: lane (cz, lx) integrates its xi row along y
// against the y table and writes the column of the tile's patch.
template <class L, int NQ, int Q>
__device__ inline void integrate_y_col(const double* xi, double* __restrict__ out, const double* __restrict__ tyt,
                                       int lane, int nt, int tx, int ty, int tz) {
    if (lane >= L::Wz * L::Wx) return;
    const int cz = lane / L::Wx, lx = lane - cz * L::Wx;
    const double* col = xi + lane * (Q + 1);
    double c[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) c[k] = col[k];
    double o[L::Wy];
#pragma unroll
    for (int ly = 0; ly < L::Wy; ++ly) o[ly] = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int le = q / NQ;
#pragma unroll
        for (int j = 0; j < L::Ky; ++j) o[le + j] = fma(tyt[q * L::Ky + j], c[q], o[le + j]);
    }
    // consecutive ly are nt * Wx apart in the patch
    double* dst = out + patch_at<L>(nt, tx, ty, tz, lx, 0, cz);
    const int pitch = nt * L::Wx;
#pragma unroll
    for (int ly = 0; ly < L::Wy; ++ly) dst[ly * pitch] = o[ly];
}

// MET = 0: the metric w_q DF^T DF / det DF is streamed from memory (any map);
// MET = 1: it is recomputed at each Gauss point for x -> x + a s(x) (1,1,1)
// with s = sin(pi x) sin(pi y) sin(pi z) (a = 0: identity), from per-axis
// tables of sin, cos and weights: DF = I + a (1,1,1)^T grad(s)^T gives
// det DF = 1 + a (g1 + g2 + g3) and (DF^T DF)_ij = d_ij + a (g_i + g_j) + 3 a^2 g_i g_j.
// WPE: minimum waves per SIMD the compiler must allow (1: its own choice; 4:
// registers capped at 128 for a fourth resident workgroup per CU).
// `tabg` and `axt` are A.tab and A.axis_tab, passed again as restrict
// parameters so that their uniform reads go through the scalar cache.
template <int P, int SPACE, bool CURL, int MET, int WPE>
__global__ void __launch_bounds__(MassCfg<P>::NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
mass_kernel(const MassArgs A, const double* __restrict__ tabg, const double* __restrict__ axt) {
    constexpr int NQ = P + 1, Q = TILE * NQ, NT = MassCfg<P>::NT;
    constexpr int SRC = CURL ? (SPACE == SP_B ? SP_E : SP_H) : SPACE;
    // 1-form spaces (the mass matrices of the first scheme): the covariant
    // factor det DF (DF^T DF)^{-1} and the material as a factor; 2-form spaces:
    // DF^T DF / det DF and the material's inverse
    constexpr bool FORM1 = SPACE == SP_E || SPACE == SP_H;
    static_assert(!(FORM1 && CURL), "the curl is fused only into the 2-form masses");
    using L0 = Lay<P, SPACE, 0>;
    using L1 = Lay<P, SPACE, 1>;
    using L2 = Lay<P, SPACE, 2>;
    using S0 = Lay<P, SRC, 0>;
    using S1 = Lay<P, SRC, 1>;
    using S2 = Lay<P, SRC, 2>;
    using P0 = MassPitch<L0, Q>;
    using P1 = MassPitch<L1, Q>;
    using P2 = MassPitch<L2, Q>;
    static_assert(NT >= 3 * 64, "parts 1a and 3b take one wave per component");
    static_assert(L0::Wz * L0::Wx <= 64 && L1::Wz * L1::Wx <= 64 && L2::Wz * L2::Wx <= 64,
                  "a component's (z, x) columns fit one wave");
    static_assert(L0::Wz * Q <= NT && L1::Wz * Q <= NT && L2::Wz * Q <= NT, "one x row per thread");
    constexpr int KMAX = P + 1;
    constexpr int TSL = TILE * NQ * KMAX;  // one table slice
    // LDS map: x and z tables (two slots each) | input windows, later the
    // z-integral planes of one component | per component: y-contracted window,
    // later x-integrated rows
    constexpr int SW = CURL ? S0::size + S1::size + S2::size : L0::size + L1::size + L2::size;
    constexpr int WZM = L0::Wz > L1::Wz ? (L0::Wz > L2::Wz ? L0::Wz : L2::Wz) : (L1::Wz > L2::Wz ? L1::Wz : L2::Wz);
    constexpr int RB = WZM * Q * (Q + 1);
    constexpr int R0 = SW > RB ? SW : RB;
    constexpr int OT = 0, OR = OT + 4 * TSL;
    constexpr int OY0 = OR + R0, OY1 = OY0 + P0::size, OY2 = OY1 + P1::size, OEND = OY2 + P2::size;
    __shared__ double sm[OEND];

    const int tid = threadIdx.x;
    const int nt = A.ntile;
    const int tile = xcd_tile(blockIdx.x, nt * nt * nt);
    const int b = blockIdx.y;
    const int tx = tile % nt, ty = (tile / nt) % nt, tz = tile / (nt * nt);
    const double* src = A.src + int64_t(b) * A.src_stride;
    const int qy = tid / Q, qx = tid % Q;
    const bool active = tid < Q * Q;
    const int wave = tid / 64, lane = tid % 64;
    // the first Gauss-point plane of the metric is requested before the window
    // set-up so that its latency overlaps it
    const double* gm = A.metric + int64_t(tile) * Q * 6 * Q * Q + qy * Q + qx;
    double g[6] = {0, 0, 0, 0, 0, 0};
    if (MET == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) g[k] = active ? __builtin_nontemporal_load(gm + k * Q * Q) : 0.0;
    }

    // ---- tracked 2-form entries owned by this tile, one wave per component
    // (requested first: the per-wave branches must not wait for other loads) ----
    constexpr int WYM = L0::Wy > L1::Wy ? (L0::Wy > L2::Wy ? L0::Wy : L2::Wy) : (L1::Wy > L2::Wy ? L1::Wy : L2::Wy);
    double* tr = (CURL && A.track) ? A.track + int64_t(b) * A.track_stride : nullptr;
    int tk[WYM];
    double tv[WYM];
    if (tr && wave == 0)
        track_column_load<L0, WYM>(tr + A.track_comp_off[0], A.track_dims[0], tx, ty, tz, nt, lane, tk, tv);
    else if (tr && wave == 1)
        track_column_load<L1, WYM>(tr + A.track_comp_off[1], A.track_dims[1], tx, ty, tz, nt, lane, tk, tv);
    else if (tr && wave == 2)
        track_column_load<L2, WYM>(tr + A.track_comp_off[2], A.track_dims[2], tx, ty, tz, nt, lane, tk, tv);

    // ---- per (x, y) column: 1/gamma (1-forms: gamma) of its four elements and, for the analytic
    // metric, q = a grad s = (a1 s_z, a2 s_z, a3 c_z) up to the z factors; read
    // here, before the column registers fill up ----
    // (analytic metric: ig[le] holds w_x w_y / gamma_e, and a12 = a1 + a2)
    // (only the loads here: the factors are formed after the windows are
    // stored, so that no wait for these loads precedes the other requests)
    double ig[TILE], ax[6] = {0, 0, 0, 0, 0, 0};
    if (active) {
        const int ex = tx * TILE + qx / NQ, ey = ty * TILE + qy / NQ;
#pragma unroll
        for (int le = 0; le < TILE; ++le)
            ig[le] = A.inv_gamma ? A.inv_gamma[(int64_t(tz * TILE + le) * A.npad + ey) * A.npad + ex] : 1.0;
        if (MET == 1) {
            const int64_t npq = int64_t(A.npad) * NQ;
            const int gxq = tx * TILE * NQ + qx, gyq = ty * TILE * NQ + qy;
            ax[0] = axt[gxq];
            ax[1] = axt[npq + gxq];
            ax[2] = axt[2 * npq + gxq];
            ax[3] = axt[gyq];
            ax[4] = axt[npq + gyq];
            ax[5] = axt[2 * npq + gyq];
        }
    }

    // ---- x and z tables of the tile: [axis x, z][slot][element][point][function] ----
    {
        constexpr int ST = (4 * TSL + NT - 1) / NT;
        // the four (axis, slot) tags are compile-time: their table offsets are
        // scalars, selected per lane (a lane-indexed read of the argument array
        // would be a vector load and a wait for every earlier request)
        constexpr int T0 = space_tag(SPACE, 0, 0), T1 = space_tag(SPACE, 1, 0);
        constexpr int T2 = space_tag(SPACE, 2, 2), T3 = space_tag(SPACE, 0, 2);
        constexpr int K0 = tag_support(P, T0), K1 = tag_support(P, T1), K2 = tag_support(P, T2), K3 = tag_support(P, T3);
        const int64_t b0 = A.tab_off[T0] + int64_t(tx) * TILE * NQ * K0, b1 = A.tab_off[T1] + int64_t(tx) * TILE * NQ * K1;
        const int64_t b2 = A.tab_off[T2] + int64_t(tz) * TILE * NQ * K2, b3 = A.tab_off[T3] + int64_t(tz) * TILE * NQ * K3;
        double r[ST];
#pragma unroll
        for (int q = 0; q < ST; ++q) {
            const int i = tid + NT * q;
            const int sel = i / TSL, k = i % TSL;  // sel = 2 az + slot
            const int K = sel == 0 ? K0 : (sel == 1 ? K1 : (sel == 2 ? K2 : K3));
            const int64_t base = sel == 0 ? b0 : (sel == 1 ? b1 : (sel == 2 ? b2 : b3));
            const bool ok = i < 4 * TSL && k < TILE * NQ * K;
            const double t = tabg[ok ? base + k : 0];
            r[q] = ok ? t : 0.0;
        }
        // ---- input windows (the 1-form when the curl is fused, else the
        // 2-form), requested before any of the LDS stores waits for a load ----
        using W0 = typename std::conditional<CURL, S0, L0>::type;
        using W1 = typename std::conditional<CURL, S1, L1>::type;
        using W2 = typename std::conditional<CURL, S2, L2>::type;
        constexpr int WG = NT / 64;
        constexpr int I0 = (W0::Wz + WG - 1) / WG, I1 = (W1::Wz + WG - 1) / WG, I2 = (W2::Wz + WG - 1) / WG;
        const int wlx = tid & 7, wly = (tid >> 3) & 7, wg = tid >> 6;
        double w0[I0], w1[I1], w2[I2];
        window_rows<P, W0, WG, I0>(w0, src + A.src_comp_off[0], A.src_dims[0], tx, ty, tz, A.n0, A.n1, wlx, wly, wg);
        window_rows<P, W1, WG, I1>(w1, src + A.src_comp_off[1], A.src_dims[1], tx, ty, tz, A.n0, A.n1, wlx, wly, wg);
        window_rows<P, W2, WG, I2>(w2, src + A.src_comp_off[2], A.src_dims[2], tx, ty, tz, A.n0, A.n1, wlx, wly, wg);
#pragma unroll
        for (int q = 0; q < ST; ++q) {
            const int i = tid + NT * q;
            if (i < 4 * TSL) sm[OT + i] = r[q];
        }
        store_rows<W0, WG, I0>(sm + OR, w0, wlx, wly, wg);
        store_rows<W1, WG, I1>(sm + OR + W0::size, w1, wlx, wly, wg);
        store_rows<W2, WG, I2>(sm + OR + W0::size + W1::size, w2, wlx, wly, wg);
    }
    // analytic metric, per (x, y) column: q = a grad s = (a1 s_z, a2 s_z, a3 c_z)
    // up to the z factors, a12 = a1 + a2, and ig[le] = w_x w_y / gamma_e
    double a1 = 0.0, a2 = 0.0, a3 = 0.0, a12 = 0.0;
    if (MET == 1 && active) {
        const double sx = ax[0], cx = ax[1], wx = ax[2], sy = ax[3], cy = ax[4], wy = ax[5];
        a1 = A.amp * M_PI * cx * sy;
        a2 = A.amp * M_PI * sx * cy;
        a3 = A.amp * M_PI * sx * sy;
        a12 = a1 + a2;
        const double wxy = wx * wy;
#pragma unroll
        for (int le = 0; le < TILE; ++le) ig[le] *= wxy;
    }
    __syncthreads();

    // ---- part 1a: y contraction of the windows, one wave per component ----
    {
        const double* s0 = sm + OR;
        const double* s1 = s0 + S0::size;
        const double* s2 = s1 + S1::size;
        const double* x0 = sm + OR;
        const double* x1 = x0 + L0::size;
        const double* x2 = x1 + L1::size;
        if (wave == 0)
            forward_y<P, SRC, SPACE, 0, CURL, NQ, Q>(s0, s1, s2, x0, sm + OY0,
                                                     axis_table<P, SPACE, 1, 1>(tabg, A.tab_off, ty), lane, tr, A,
                                                     tk, tv);
        else if (wave == 1)
            forward_y<P, SRC, SPACE, 1, CURL, NQ, Q>(s0, s1, s2, x1, sm + OY1,
                                                     axis_table<P, SPACE, 1, 0>(tabg, A.tab_off, ty), lane, tr, A,
                                                     tk, tv);
        else if (wave == 2)
            forward_y<P, SRC, SPACE, 2, CURL, NQ, Q>(s0, s1, s2, x2, sm + OY2,
                                                     axis_table<P, SPACE, 1, 1>(tabg, A.tab_off, ty), lane, tr, A,
                                                     tk, tv);
    }
    __syncthreads();

    // ---- part 1b: x contraction into the register columns ----
    double A0[L0::Wz], A1[L1::Wz], A2[L2::Wz];
    if (active) {
        // one component at a time: the scheduler would otherwise hoist all
        // three components' LDS reads and run out of registers
        forward_x<L0, NQ, Q>(sm + OY0, sm + OT, A0, qy, qx);
        __builtin_amdgcn_sched_barrier(0);
        forward_x<L1, NQ, Q>(sm + OY1, sm + OT + TSL, A1, qy, qx);
        __builtin_amdgcn_sched_barrier(0);
        forward_x<L2, NQ, Q>(sm + OY2, sm + OT + TSL, A2, qy, qx);
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- part 2: stream the Gauss-point planes: z contraction, metric, z integral ----
    double R0c[L0::Wz], R1c[L1::Wz], R2c[L2::Wz];
#pragma unroll
    for (int k = 0; k < L0::Wz; ++k) R0c[k] = 0.0;
#pragma unroll
    for (int k = 0; k < L1::Wz; ++k) R1c[k] = 0.0;
#pragma unroll
    for (int k = 0; k < L2::Wz; ++k) R2c[k] = 0.0;
    if (active) {
        const double* tz0 = sm + OT + 3 * TSL;  // components 0 and 1 are across z
        const double* tz2 = sm + OT + 2 * TSL;  // component 2 is along z
        const int64_t npq = int64_t(A.npad) * NQ;
#pragma unroll
        for (int le = 0; le < TILE; ++le) {
#pragma unroll
            for (int iq = 0; iq < NQ; ++iq) {
                const int qz = le * NQ + iq;
                double gn[6];  // next plane in flight while this one is used
                if (MET == 0 && qz + 1 < Q) {
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        gn[k] = __builtin_nontemporal_load(gm + int64_t(qz + 1) * 6 * Q * Q + k * Q * Q);
                }
                // analytic metric: with q = a grad s, DF = I + 1 q^T, det DF = 1 + q.1 and
                // w DF^T DF / det DF = f (I + q 1^T + 1 q^T + 3 q q^T), f = w / det DF,
                // applied below as a rank-2 update of the identity
                double q1 = 0.0, q2 = 0.0, q3 = 0.0, sf = 0.0, dd = 1.0, rd = 1.0;
                if (MET == 1) {
                    const int gzq = tz * TILE * NQ + qz;
                    const double sz = axt[gzq], cz = axt[npq + gzq], wz = axt[2 * npq + gzq];
                    q1 = a1 * sz;
                    q2 = a2 * sz;
                    q3 = a3 * cz;
                    // det DF = 1 + (a1 + a2) s_z + a3 c_z
                    dd = fma(a12, sz, fma(a3, cz, 1.0));
                    rd = recip_nr(dd);
                    // 2-form: s f = (w / gamma_e) / det DF; 1-form: w gamma_e
                    sf = FORM1 ? ig[le] * wz : (ig[le] * wz) * rd;
                }
                const double* t0 = tz0 + qz * L0::Kz;
                const double* t2 = tz2 + qz * L2::Kz;
                double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
                for (int j = 0; j < L0::Kz; ++j) v0 += t0[j] * A0[le + j];
#pragma unroll
                for (int j = 0; j < L1::Kz; ++j) v1 += t0[j] * A1[le + j];
#pragma unroll
                for (int j = 0; j < L2::Kz; ++j) v2 += t2[j] * A2[le + j];
                double u0, u1, u2;
                if (MET == 1 && FORM1) {
                    // DF^{-1} = I - 1 q^T / d (d = det DF), so
                    // det DF (DF^T DF)^{-1} v = d v - S q + (|q|^2 S / d - Q) 1,
                    // S = sum v, Q = q . v, scaled by sf = w gamma_e
                    const double Sv = v0 + v1 + v2, Qv = fma(q1, v0, fma(q2, v1, q3 * v2));
                    const double qq = fma(q1, q1, fma(q2, q2, q3 * q3));
                    const double sd = sf * dd, ss = -sf * Sv, c1 = sf * fma(qq * Sv, rd, -Qv);
                    u0 = fma(sd, v0, fma(ss, q1, c1));
                    u1 = fma(sd, v1, fma(ss, q2, c1));
                    u2 = fma(sd, v2, fma(ss, q3, c1));
                } else if (MET == 1) {
                    // G v = f (v + (S + 3 Q) q + Q 1), S = sum v, Q = q . v, as
                    // u = sf v + (sf (S + 3 Q)) q + sf Q 1
                    const double Qv = fma(q1, v0, fma(q2, v1, q3 * v2));
                    const double cq = sf * fma(3.0, Qv, v0 + v1 + v2), bq = sf * Qv;
                    u0 = fma(sf, v0, fma(cq, q1, bq));
                    u1 = fma(sf, v1, fma(cq, q2, bq));
                    u2 = fma(sf, v2, fma(cq, q3, bq));
                } else {
                    const double s = ig[le];
                    u0 = s * (g[0] * v0 + g[3] * v1 + g[4] * v2);
                    u1 = s * (g[3] * v0 + g[1] * v1 + g[5] * v2);
                    u2 = s * (g[4] * v0 + g[5] * v1 + g[2] * v2);
                }
#pragma unroll
                for (int j = 0; j < L0::Kz; ++j) R0c[le + j] += t0[j] * u0;
#pragma unroll
                for (int j = 0; j < L1::Kz; ++j) R1c[le + j] += t0[j] * u1;
#pragma unroll
                for (int j = 0; j < L2::Kz; ++j) R2c[le + j] += t2[j] * u2;
                if (MET == 0 && qz + 1 < Q) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) g[k] = gn[k];
                }
            }
        }
    }

    // ---- part 3: x integrals row by row (R planes in the window region, last
    // read in part 1a), then y integrals, one wave per component ----
    double* rb = sm + OR;
    if (active) {
#pragma unroll
        for (int cz = 0; cz < L0::Wz; ++cz) rb[(cz * Q + qy) * (Q + 1) + qx] = R0c[cz];
    }
    __syncthreads();
    integrate_x_row<L0, NQ, Q>(rb, sm + OY0, axis_table<P, SPACE, 0, 0>(tabg, A.tab_off, tx), tid);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int cz = 0; cz < L1::Wz; ++cz) rb[(cz * Q + qy) * (Q + 1) + qx] = R1c[cz];
    }
    __syncthreads();
    integrate_x_row<L1, NQ, Q>(rb, sm + OY1, axis_table<P, SPACE, 0, 1>(tabg, A.tab_off, tx), tid);
    __syncthreads();
    if (active) {
#pragma unroll
        for (int cz = 0; cz < L2::Wz; ++cz) rb[(cz * Q + qy) * (Q + 1) + qx] = R2c[cz];
    }
    __syncthreads();
    integrate_x_row<L2, NQ, Q>(rb, sm + OY2, axis_table<P, SPACE, 0, 1>(tabg, A.tab_off, tx), tid);
    __syncthreads();
    double* out = A.patch + int64_t(b) * A.patch_stride;
    if (wave == 0)
        integrate_y_col<L0, NQ, Q>(sm + OY0, out + A.patch_comp_off[0], axis_table<P, SPACE, 1, 1>(tabg, A.tab_off, ty),
                                   lane, nt, tx, ty, tz);
    else if (wave == 1)
        integrate_y_col<L1, NQ, Q>(sm + OY1, out + A.patch_comp_off[1], axis_table<P, SPACE, 1, 0>(tabg, A.tab_off, ty),
                                   lane, nt, tx, ty, tz);
    else if (wave == 2)
        integrate_y_col<L2, NQ, Q>(sm + OY2, out + A.patch_comp_off[2], axis_table<P, SPACE, 1, 1>(tabg, A.tab_off, ty),
                                   lane, nt, tx, ty, tz);
}

// One launch of a mass kernel; with profiling events, through
// hipExtLaunchKernelGGL, which stamps them with the kernel's own start and
// end (profiling runs are never captured into graphs)
template <class K>
static void launch_mass_k(K kernel, const MassArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    if (a.prof_start && a.prof_stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a.prof_start, a.prof_stop, 0, a, a.tab, a.axis_tab);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, a, a.tab, a.axis_tab);
}

template <int P, int SPACE, bool CURL>
static void launch_mass_t(const MassArgs& a, dim3 grid, hipStream_t s) {
    // the four-wave variant exists for p <= 3 (p = 4 would spill)
    const bool w4 = a.waves4 && P <= 3;
    const dim3 block(MassCfg<P>::NT);
    if (a.metric_mode == 1) {
        if (w4) launch_mass_k(mass_kernel<P, SPACE, CURL, 1, (P <= 3 ? 4 : 1)>, a, grid, block, s);
        else launch_mass_k(mass_kernel<P, SPACE, CURL, 1, 1>, a, grid, block, s);
    } else {
        if (w4) launch_mass_k(mass_kernel<P, SPACE, CURL, 0, (P <= 3 ? 4 : 1)>, a, grid, block, s);
        else launch_mass_k(mass_kernel<P, SPACE, CURL, 0, 1>, a, grid, block, s);
    }
}

void launch_mass(int p, int space, bool curl, const MassArgs& a, int batch, hipStream_t s) {
    const int nt3 = a.ntile * a.ntile * a.ntile;
    dim3 grid(nt3, batch);
#define LM(PP)                                                                      \
    if (p == PP) {                                                                  \
        if (space == SP_B) {                                                        \
            if (curl) launch_mass_t<PP, SP_B, true>(a, grid, s);                    \
            else launch_mass_t<PP, SP_B, false>(a, grid, s);                        \
        } else if (space == SP_D) {                                                 \
            if (curl) launch_mass_t<PP, SP_D, true>(a, grid, s);                    \
            else launch_mass_t<PP, SP_D, false>(a, grid, s);                        \
        } else if (space == SP_E) {                                                 \
            launch_mass_t<PP, SP_E, false>(a, grid, s);                             \
        } else {                                                                    \
            launch_mass_t<PP, SP_H, false>(a, grid, s);                             \
        }                                                                           \
        return;                                                                     \
    }
    LM(2) LM(3) LM(4)
#undef LM
}

// ===========================================================================
// Patch gather: y_i = sum of the tile patches covering basis function i, in a
// fixed order (tiles by increasing z, y, x).  One thread per output; the
// windows are compile-time per component, the candidate tiles come from shifts.
// ===========================================================================
// q = n / d and r = n % d for 0 <= n < 2^24, d > 0, without the software
// integer division: the hardware reciprocal, refined by one Newton step, gives
// a quotient that is off by at most one, which one comparison corrects.
__device__ inline int fast_divmod(int n, int d, int& r) {
    const double dd = double(d);
    double inv = __builtin_amdgcn_rcp(dd);
    inv = fma(inv, fma(-dd, inv, 1.0), inv);
    int q = int(double(n) * inv);
    r = n - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
    return q;
}

template <int P, int SPACE>
__global__ void __launch_bounds__(256) gather_kernel(const GatherArgs A, int64_t n) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;  // fields hold fewer than 2^24 entries
    if (i >= n) return;
    const int c = i >= A.comp_off[2] ? 2 : (i >= A.comp_off[1] ? 1 : 0);
    const int li = i - int(A.comp_off[c]);
    const int nx = A.dims[c][2], ny = A.dims[c][1];
    int x, y;
    const int row = fast_divmod(li, nx, x);
    const int z = fast_divmod(row, ny, y);
    const double* patch = A.patch + int64_t(b) * A.patch_stride + A.patch_comp_off[c];
    double v;
    if (c == 0) v = gather_one<P, SPACE, 0>(patch, A.ntile, z, y, x);
    else if (c == 1) v = gather_one<P, SPACE, 1>(patch, A.ntile, z, y, x);
    else v = gather_one<P, SPACE, 2>(patch, A.ntile, z, y, x);
    A.out[int64_t(b) * A.out_stride + i] = v;
    if (A.acc) {
        double* w = A.acc + int64_t(b) * A.acc_stride + i;
        *w = fma(A.acc_alpha, v, *w);
    }
}

void launch_gather(int p, int space, const GatherArgs& a, int64_t n, int batch, hipStream_t s) {
    dim3 grid(unsigned((n + 255) / 256), batch);
#define LG(PP)                                                                                         \
    if (p == PP) {                                                                                     \
        if (space == SP_D) hipLaunchKernelGGL((gather_kernel<PP, SP_D>), grid, dim3(256), 0, s, a, n); \
        else if (space == SP_B) hipLaunchKernelGGL((gather_kernel<PP, SP_B>), grid, dim3(256), 0, s, a, n); \
        else if (space == SP_E) hipLaunchKernelGGL((gather_kernel<PP, SP_E>), grid, dim3(256), 0, s, a, n); \
        else hipLaunchKernelGGL((gather_kernel<PP, SP_H>), grid, dim3(256), 0, s, a, n);               \
        return;                                                                                        \
    }
    LG(2) LG(3) LG(4)
#undef LG
}

// ===========================================================================
// Pairing solves and applies (eqs. (4.2)-(4.5)): block c of K1 or K~1 is
// A_z (x) A_y (x) A_x, so K^{-1} applies A_x^{-1}, A_y^{-1}, A_z^{-1} along the
// lines of each axis (and K applies A_x, A_y, A_z).  Each 1D solve is a banded
// forward/backward substitution with precomputed LU factors (half bandwidth
// W = p-1), each 1D apply a banded product; the factors of a line are staged
// in LDS, shared by all lines of the workgroup.
// ===========================================================================
// Largest line handled (N <= 72 elements, p <= 4) and the LDS size of one
// staged factor set [L (n W) | U (n W) | dinv (n) | band (n (2W+1))].
constexpr int KMX_LINE_MAX = 76;
constexpr int FACTOR_MAX = 2 * KMX_LINE_MAX * 7;

// Forward/backward substitution along one line.  The dependency chain runs
// through registers only: the line values and factor coefficients of a block
// of D steps are loaded together (one wait per block), then the D steps of the
// chain run without touching memory except for the stores.
template <int W>
__device__ inline void band_solve_line(double* v, int n, int stride, const double* __restrict__ L,
                                       const double* __restrict__ U, const double* __restrict__ dinv) {
    constexpr int D = 8;
    double prev[W];
#pragma unroll
    for (int m = 0; m < W; ++m) prev[m] = 0.0;
    for (int i0 = 0; i0 < n; i0 += D) {
        double xv[D], lc[D][W];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int i = i0 + k < n ? i0 + k : n - 1;
            xv[k] = v[i * stride];
#pragma unroll
            for (int m = 0; m < W; ++m) lc[k][m] = L[i * W + m];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (i0 + k < n) {
                double s = xv[k];
#pragma unroll
                for (int m = 0; m < W; ++m) s -= lc[k][m] * prev[m];
#pragma unroll
                for (int m = W - 1; m > 0; --m) prev[m] = prev[m - 1];
                prev[0] = s;
                v[(i0 + k) * stride] = s;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < W; ++m) prev[m] = 0.0;
    for (int i0 = n - 1; i0 >= 0; i0 -= D) {
        double xv[D], uc[D][W], dc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int i = i0 - k >= 0 ? i0 - k : 0;
            xv[k] = v[i * stride];
            dc[k] = dinv[i];
#pragma unroll
            for (int m = 0; m < W; ++m) uc[k][m] = U[i * W + m];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (i0 - k >= 0) {
                double s = xv[k];
#pragma unroll
                for (int m = 0; m < W; ++m) s -= uc[k][m] * prev[m];
                s *= dc[k];
#pragma unroll
                for (int m = W - 1; m > 0; --m) prev[m] = prev[m - 1];
                prev[0] = s;
                v[(i0 - k) * stride] = s;
            }
        }
    }
}

// banded product of one output: sum_k band[i][k] x_{i-W+k} (the band holds
// zeros outside the matrix, so clamped indices contribute nothing)
template <int W>
__device__ inline double band_row(const double* x, int n, int stride, const double* __restrict__ band, int i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * W + 1; ++k) {
        int j = i - W + k;
        j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
        s += band[i * (2 * W + 1) + k] * x[j * stride];
    }
    return s;
}

// One factor set [L | U | dinv | band] (2n(2W+1) doubles) into LDS by a
// workgroup of 256 threads: every load of a thread is issued before its first
// store (one memory latency instead of one per element).
template <int W>
__device__ inline void stage_factor(double* dst, const double* __restrict__ fac, int64_t off, int n, int tid) {
    constexpr int S = (FACTOR_MAX + 255) / 256;
    const int len = 2 * n * (2 * W + 1);
    double r[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int i = tid + 256 * q;
        r[q] = i < len ? fac[off + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int i = tid + 256 * q;
        if (i < len) dst[i] = r[q];
    }
}

template <int P>
__global__ void __launch_bounds__(256) xy_kernel(const XYArgs A) {
    constexpr int W = P - 1;
    constexpr int SLOTS = (KMX_LINE_MAX * KMX_LINE_MAX + 255) / 256;
    extern __shared__ double plane[];
    __shared__ double fx[FACTOR_MAX], fy[FACTOR_MAX];
    const int c = blockIdx.y, b = blockIdx.z, iz = blockIdx.x;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    if (iz >= nz) return;
    const int nxp = nx | 1;  // odd row stride: the lines along x hit distinct LDS banks
    const int tid = threadIdx.x;
    if (A.solve) {
        stage_factor<W>(fx, A.fac, A.fac_off[A.fac_id[c][0]], nx, tid);
        stage_factor<W>(fy, A.fac, A.fac_off[A.fac_id[c][1]], ny, tid);
    }
    {
        // stage the plane: rows over the 4 waves, x over the 64 lanes
        const int lane = tid & 63, wv = tid >> 6;
        const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
        constexpr int RY = (KMX_LINE_MAX + 3) / 4;  // rows per wave
        double r0[RY], r1[RY];
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int y = wv + 4 * k;
            r0[k] = (y < ny && lane < nx) ? in[y * nx + lane] : 0.0;
            r1[k] = (y < ny && lane + 64 < nx) ? in[y * nx + lane + 64] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int y = wv + 4 * k;
            if (y < ny && lane < nx) plane[y * nxp + lane] = r0[k];
            if (y < ny && lane + 64 < nx) plane[y * nxp + lane + 64] = r1[k];
        }
    }
    __syncthreads();
    // point sources: subtract g(t) s on this plane, in a fixed order
    if (A.n_src > 0) {
        if (tid == 0) {
            for (int k = A.src_off[b]; k < A.src_off[b + 1]; ++k) {
                const double* pr = A.src_prof + 4 * k;
                const double dtt = (A.t_dev ? *A.t_dev : 0.0) + A.t_src - pr[0];
                const double gt = pr[2] * exp(-dtt * dtt / (2.0 * pr[1] * pr[1]));
                const double* en = A.src_entries + int64_t(k) * A.entries_per * 5;
                for (int e = 0; e < A.entries_per; ++e) {
                    if (int(en[5 * e]) != c || int(en[5 * e + 1]) != iz) continue;
                    plane[int(en[5 * e + 2]) * nxp + int(en[5 * e + 3])] -= gt * en[5 * e + 4];
                }
            }
        }
        __syncthreads();
    }
    if (A.solve == 1) {
        for (int y = tid; y < ny; y += 256) band_solve_line<W>(plane + y * nxp, nx, 1, fx, fx + nx * W, fx + 2 * nx * W);
        __syncthreads();
        for (int x = tid; x < nx; x += 256) band_solve_line<W>(plane + x, ny, nxp, fy, fy + ny * W, fy + 2 * ny * W);
        __syncthreads();
    } else if (A.solve == 2) {
        // every output of a banded product is independent: compute all of a
        // direction into registers, then write back
        const double* bx = fx + 2 * nx * W + nx;
        const double* by = fy + 2 * ny * W + ny;
        double r[SLOTS];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int i = tid + s * 256;
            if (i < nx * ny) r[s] = band_row<W>(plane + (i / nx) * nxp, nx, 1, bx, i % nx);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int i = tid + s * 256;
            if (i < nx * ny) plane[(i / nx) * nxp + (i % nx)] = r[s];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int i = tid + s * 256;
            if (i < nx * ny) r[s] = band_row<W>(plane + (i % nx), ny, nxp, by, i / nx);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int i = tid + s * 256;
            if (i < nx * ny) plane[(i / nx) * nxp + (i % nx)] = r[s];
        }
        __syncthreads();
    }
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c] + int64_t(iz) * nx * ny;
    {
        const int lane = tid & 63, wv = tid >> 6;
        for (int y = wv; y < ny; y += 4) {
            if (lane < nx) out[y * nx + lane] = plane[y * nxp + lane];
            if (lane + 64 < nx) out[y * nx + lane + 64] = plane[y * nxp + lane + 64];
        }
    }
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
#define LX(PP)                                                                         \
    if (p == PP) {                                                                     \
        hipLaunchKernelGGL((xy_kernel<PP>), grid, dim3(256), shm, s, a);               \
        return;                                                                        \
    }
    LX(2) LX(3) LX(4)
#undef LX
}

// z solve / apply: 64 (x, y) columns per workgroup staged in LDS by all 256
// threads (coalesced rows), one thread per column for the substitution (the
// banded apply uses all threads), then the fused update
// out = (accumulate ? out : 0) + alpha x.
template <int P>
__global__ void __launch_bounds__(256) z_kernel(const ZArgs A) {
    constexpr int W = P - 1;
    constexpr int SLOTS = (KMX_LINE_MAX + 3) / 4;
    extern __shared__ double col[];  // [nz][64]
    __shared__ double f[FACTOR_MAX];
    const int c = blockIdx.y, b = blockIdx.z;
    const int nz = A.dims[c][0], ny = A.dims[c][1], nx = A.dims[c][2];
    const int64_t ncol = int64_t(nx) * ny;
    const int64_t col0 = int64_t(blockIdx.x) * 64;
    if (col0 >= ncol) return;
    const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
    const int64_t colid = col0 + lane;
    const bool ok = colid < ncol;
    if (A.solve) stage_factor<W>(f, A.fac, A.fac_off[A.fac_id[c]], nz, tid);
    const double* in = A.in + int64_t(b) * A.in_stride + A.comp_off[c];
    double* out = A.out + int64_t(b) * A.out_stride + A.comp_off[c];
    {
        double r[SLOTS];  // all loads of this thread in flight at once
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int z = grp + 4 * s;
            r[s] = (ok && z < nz) ? in[int64_t(z) * ncol + colid] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int z = grp + 4 * s;
            if (z < nz) col[z * 64 + lane] = r[s];
        }
    }
    __syncthreads();
    if (A.solve == 1) {
        if (grp == 0) band_solve_line<W>(col + lane, nz, 64, f, f + nz * W, f + 2 * nz * W);
        __syncthreads();
    } else if (A.solve == 2) {
        const double* band = f + 2 * nz * W + nz;
        double r[SLOTS];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int z = grp + 4 * s;
            if (z < nz) r[s] = band_row<W>(col + lane, nz, 64, band, z);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int z = grp + 4 * s;
            if (z < nz) col[z * 64 + lane] = r[s];
        }
        __syncthreads();
    }
    if (!ok) return;
    const double alpha = A.alpha;
    if (A.accumulate) {
        double o[SLOTS];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int z = grp + 4 * s;
            o[s] = z < nz ? out[int64_t(z) * ncol + colid] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int z = grp + 4 * s;
            if (z < nz) out[int64_t(z) * ncol + colid] = o[s] + alpha * col[z * 64 + lane];
        }
    } else {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int z = grp + 4 * s;
            if (z < nz) out[int64_t(z) * ncol + colid] = alpha * col[z * 64 + lane];
        }
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
        hipLaunchKernelGGL((z_kernel<PP>), grid, dim3(256), shm, s, a);       \
        return;                                                               \
    }
    LZ(2) LZ(3) LZ(4)
#undef LZ
}

// ===========================================================================
// Curl (incidence matrices, Section 2.4): out = beta out + alpha (d_{c+1} u_{c+2}
// - d_{c+2} u_{c+1}); primal d: v[k] - v[k-1] (zero outside), dual d~: v[r+1] - v[r].
// ===========================================================================
// the same for the primal difference, branch-free: every load comes from an
// index clamped inside the component and out-of-range taps are selected away
__device__ inline double diff1_primal(const double* u, const int d[3], int axis, int z, int y, int x) {
    const int n = d[2 - axis];
    const int k = axis == 0 ? x : (axis == 1 ? y : z);
    const int stride = axis == 0 ? 1 : (axis == 1 ? d[2] : d[1] * d[2]);
    const int base = (z * d[1] + y) * d[2] + x;
    const int k1 = k < n - 1 ? k : n - 1;
    const int k0 = k - 1 < 0 ? 0 : (k - 1 < n - 1 ? k - 1 : n - 1);
    const double a = u[base + (k1 - k) * stride];
    const double c = u[base + (k0 - k) * stride];
    return (k < n ? a : 0.0) - (k - 1 >= 0 && k - 1 < n ? c : 0.0);
}

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
// Energies (3.2) and the leapfrog invariant, FP64, deterministic tree sums:
//   term0 = d . (K1 e)  over X~^2
//   term1 = b . (K~1 h), term2 = (K~1 h) . (D^1 e)  over X^2_{h,0}
// ===========================================================================
// Sum of three values over a workgroup of NTH threads in a fixed order: a
// butterfly within each wave, then the wave partials in wave order (one
// barrier).  out is written by thread 0.
template <int NTH>
__device__ inline void block_sum3(double v0, double v1, double v2, double* out) {
    constexpr int NW = NTH / 64;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        v0 += __shfl_xor(v0, m, 64);
        v1 += __shfl_xor(v1, m, 64);
        v2 += __shfl_xor(v2, m, 64);
    }
    __shared__ double s[3][NW];
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s[0][w] = v0;
        s[1][w] = v1;
        s[2][w] = v2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = s[0][0], t1 = s[1][0], t2 = s[2][0];
#pragma unroll
        for (int k = 1; k < NW; ++k) {
            t0 += s[0][k];
            t1 += s[1][k];
            t2 += s[2][k];
        }
        out[0] = t0;
        out[1] = t1;
        out[2] = t2;
    }
}

// Fused energy terms: one workgroup per (component, pair of z planes, block
// of EROWS rows) forms w = K v on its rows (K1 e for the first term, K~1 h for
// the other two) by the Kronecker structure: the z band combines 2W+1 planes
// (the 2W+2 planes staged once serve both output planes), then the x and y
// bands run in LDS; the dot products with d (first term), b and D^1 e (second
// and third) follow in the same pass.  Blocks [0, nb0) do the first term,
// [nb0, nb0 + nb1) the others; each writes its three partial sums (zeros for
// terms it does not own) for the fixed-order final sum.
constexpr int EROWS = 16;
constexpr int EPLANES = 2;  // output planes per workgroup

template <int P>
__global__ void __launch_bounds__(256) energy_fused_kernel(const EnergyFusedArgs A) {
    constexpr int W = P - 1, B = 2 * W + 1;
    constexpr int TR = EROWS + 2 * W;  // staged rows (with the y halo)
    constexpr int ZL = B + EPLANES - 1;  // staged planes
    __shared__ double tile[EPLANES][TR * KMX_LINE_MAX];
    __shared__ double band[3][KMX_LINE_MAX * B];
    const int tid = threadIdx.x, bm = blockIdx.y;
    // XCD-aware order: each XCD takes a contiguous range of (component, plane
    // pair, row block), so the planes that neighbouring blocks share stay in its L2
    const int blk = xcd_tile(blockIdx.x, A.nb[0] + A.nb[1]);
    const int mode = blk < A.nb[0] ? 0 : 1;
    int rem = mode == 0 ? blk : blk - A.nb[0];
    int c = 0;
    while (c < 2 && rem >= A.cb[mode][c]) rem -= A.cb[mode][c++];
    const int* d = mode == 0 ? A.e_dims[c] : A.h_dims[c];
    const int nz = d[0], ny = d[1], nx = d[2];
    const int nyb = (ny + EROWS - 1) / EROWS;
    const int z0 = (rem / nyb) * EPLANES, y0 = (rem % nyb) * EROWS;
    const double* E = A.E + int64_t(bm) * 2 * A.n_e;
    const double* H = A.H + int64_t(bm) * 2 * A.n_h;
    const double* v = (mode == 0 ? E + A.e_comp_off[c] : H + A.h_comp_off[c]);
    // bands of the three axes (the factor sets' stored matrix), all loads first
    {
        constexpr int SB = (KMX_LINE_MAX * B + 255) / 256;
        double r[3][SB];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int n = d[2 - a];
            const double* src = A.fac + A.fac_off[A.fac_id[mode][c][a]] + 2 * int64_t(n) * W + n;
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                // branch-free: load from an index inside the array, then select
                const int i = tid + 256 * q;
                const double t = src[i < n * B ? i : 0];
                r[a][q] = i < n * B ? t : 0.0;
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int n = d[2 - a];
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                const int i = tid + 256 * q;
                if (i < n * B) band[a][i] = r[a][q];
            }
        }
    }
    __syncthreads();
    // z band: tile[j][r][x] = sum_k Kz(z0+j, z0+j-W+k) v[z0+j-W+k][y0-W+r][x];
    // every load of a thread is issued before the first is used
    constexpr int SL = (TR * KMX_LINE_MAX + 255) / 256;
    {
        double vz[SL][ZL];
#pragma unroll
        for (int q = 0; q < SL; ++q) {
            const int i = tid + q * 256, r = i / nx, x = i % nx, y = y0 - W + r;
#pragma unroll
            for (int k = 0; k < ZL; ++k) {
                const int zz = z0 - W + k;
                const bool ok = i < TR * nx && y >= 0 && y < ny && zz >= 0 && zz < nz;
                const double t = v[ok ? (zz * ny + y) * nx + x : 0];
                vz[q][k] = ok ? t : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < EPLANES; ++j) {
            // a plane past the field has a zero band row (its outputs are not used)
            const int zj = z0 + j < nz ? z0 + j : nz - 1;
            const double bw = z0 + j < nz ? 1.0 : 0.0;
#pragma unroll
            for (int q = 0; q < SL; ++q) {
                const int i = tid + q * 256;
                if (i < TR * nx) {
                    double s = 0.0;
#pragma unroll
                    for (int k = 0; k < B; ++k) s += band[2][zj * B + k] * vz[q][k + j];
                    tile[j][(i / nx) * KMX_LINE_MAX + (i % nx)] = bw * s;
                }
            }
        }
    }
    __syncthreads();
    // x band, row by row (outputs to registers first: the rows are updated in place)
    double t[EPLANES][SL];
#pragma unroll
    for (int j = 0; j < EPLANES; ++j)
#pragma unroll
        for (int q = 0; q < SL; ++q) {
            const int i = tid + q * 256;
            t[j][q] = 0.0;
            if (i < TR * nx) {
                const int r = i / nx, x = i % nx;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    // the band is zero outside the matrix: a clamped index adds nothing
                    int xx = x - W + k;
                    xx = xx < 0 ? 0 : (xx > nx - 1 ? nx - 1 : xx);
                    t[j][q] += band[0][x * B + k] * tile[j][r * KMX_LINE_MAX + xx];
                }
            }
        }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EPLANES; ++j)
#pragma unroll
        for (int q = 0; q < SL; ++q) {
            const int i = tid + q * 256;
            if (i < TR * nx) tile[j][(i / nx) * KMX_LINE_MAX + (i % nx)] = t[j][q];
        }
    __syncthreads();
    // y band on the owned rows, then the dot products (partner loads first)
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int rows = ny - y0 < EROWS ? ny - y0 : EROWS;
    constexpr int SO = (EROWS * KMX_LINE_MAX + 255) / 256;
    double pb[EPLANES][SO], pc[EPLANES][SO];
#pragma unroll
    for (int j = 0; j < EPLANES; ++j)
#pragma unroll
        for (int q = 0; q < SO; ++q) {
            const int i = tid + q * 256, z = z0 + j;
            pb[j][q] = pc[j][q] = 0.0;
            if (i < rows * nx && z < nz) {
                const int y = y0 + i / nx, x = i % nx;
                const int64_t at = (int64_t(z) * ny + y) * nx + x;
                if (mode == 0) {
                    pb[j][q] = E[A.n_e + A.e_comp_off[c] + at];
                } else {
                    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
                    pb[j][q] = H[A.n_h + A.h_comp_off[c] + at];
                    pc[j][q] = diff1_primal(E + A.e_comp_off[a2], A.e_dims[a2], a1, z, y, x) -
                               diff1_primal(E + A.e_comp_off[a1], A.e_dims[a1], a2, z, y, x);
                }
            }
        }
#pragma unroll
    for (int j = 0; j < EPLANES; ++j)
#pragma unroll
        for (int q = 0; q < SO; ++q) {
            const int i = tid + q * 256;
            if (i < rows * nx && z0 + j < nz) {
                const int ry = i / nx, x = i % nx, y = y0 + ry;
                double w = 0.0;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    // rows of the tile outside the field hold finite values and
                    // meet zero band entries
                    w += band[1][y * B + k] * tile[j][(ry + k) * KMX_LINE_MAX + x];
                }
                if (mode == 0) {
                    s0 += w * pb[j][q];
                } else {
                    s1 += w * pb[j][q];
                    s2 += w * pc[j][q];
                }
            }
        }
    __shared__ double r[3];
    block_sum3<256>(s0, s1, s2, r);
    if (tid == 0) {
        double* o = A.partial + (int64_t(bm) * (A.nb[0] + A.nb[1]) + blk) * 3;
        o[0] = r[0];
        o[1] = r[1];
        o[2] = r[2];
    }
}

void launch_energy_fused(int p, const EnergyFusedArgs& a, int batch, hipStream_t s) {
    dim3 grid(a.nb[0] + a.nb[1], batch);
#define LE(PP)                                                                      \
    if (p == PP) {                                                                  \
        hipLaunchKernelGGL((energy_fused_kernel<PP>), grid, dim3(256), 0, s, a);    \
        return;                                                                     \
    }
    LE(2) LE(3) LE(4)
#undef LE
}

int energy_fused_blocks(const int dims[3][3], int cb[3]) {
    int tot = 0;
    for (int c = 0; c < 3; ++c) {
        cb[c] = ((dims[c][0] + EPLANES - 1) / EPLANES) * ((dims[c][1] + EROWS - 1) / EROWS);
        tot += cb[c];
    }
    return tot;
}

// Energy terms from the kept images w_e = K1 e and w_h = K~1 h (the step
// updates them with the gathered mass applies: K~1 h^{n+1/2} = K~1 h^{n-1/2}
// - dt M D^1 e^n and K1 e^{n+1} = K1 e^n + dt M~ D~^1 h^{n+1/2}, the Hodge
// relations of eqs. (3.11) and (3.13) applied to the increments): per block
// the partial sums of d . w_e, b . w_h and w_h . D^1 e, in a fixed order
// (grid-stride loops over a fixed grid, then block_sum3).  The first EB
// working blocks take the d . w_e items, the others the b . w_h and
// w_h . D^1 e items by 2-form positions.  Block 0 takes no items:
// with A.prev_out set it sums the previous step's partials into that step's
// energy (what energy_final_kernel does), so that a run of steps needs the
// separate final launch only after its last step.  The grid stays at
// ENERGY_DOT_BLOCKS, which fills the chip's workgroup slots in one wave.
__device__ inline void energy_finish(const double* partial, int nblocks, double dt, double* out) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += 256) {
        t0 += partial[int64_t(k) * 3];
        t1 += partial[int64_t(k) * 3 + 1];
        t2 += partial[int64_t(k) * 3 + 2];
    }
    __shared__ double r[3];
    block_sum3<256>(t0, t1, t2, r);
    __syncthreads();
    if (threadIdx.x == 0) *out = 0.5 * (r[0] + r[1]) - 0.5 * dt * r[2];
}

// One e component's value at (z, y, x) and at the positions one step back
// along its two other axes (zero outside the component: e is zero on the
// boundary), the three loads issued together.
template <int A_>
__device__ inline void e_star(const double* u, const int d[3], int z, int y, int x, double& c, double& m1,
                              double& m2) {
    constexpr int a1 = (A_ + 1) % 3, a2 = (A_ + 2) % 3;  // the axes it is differenced along
    const int nz = d[0], ny = d[1], nx = d[2];
    const int base = (z * ny + y) * nx + x;
    auto back = [&](int ax) { return ax == 0 ? 1 : (ax == 1 ? nx : nx * ny); };
    auto coord = [&](int ax) { return ax == 0 ? x : (ax == 1 ? y : z); };
    const bool in = z < nz && y < ny && x < nx;
    const bool in1 = coord(a1) >= 1 && coord(a1) - 1 < d[2 - a1] && (a1 == 2 || z < nz) &&
                     (a1 == 1 || y < ny) && (a1 == 0 || x < nx);
    const bool in2 = coord(a2) >= 1 && coord(a2) - 1 < d[2 - a2] && (a2 == 2 || z < nz) &&
                     (a2 == 1 || y < ny) && (a2 == 0 || x < nx);
    const double v = u[in ? base : 0], v1 = u[in1 ? base - back(a1) : 0], v2 = u[in2 ? base - back(a2) : 0];
    c = in ? v : 0.0;
    m1 = in1 ? v1 : 0.0;
    m2 = in2 ? v2 : 0.0;
}

template <int U, int EB>
__global__ void __launch_bounds__(256) energy_dots_kernel(const EnergyDotsArgs A) {
    const int bm = blockIdx.y;
    constexpr int NB = ENERGY_DOT_WORKERS;
    if (blockIdx.x == 0) {
        if (A.prev_out) energy_finish(A.prev_partial + int64_t(bm) * NB * 3, NB, A.prev_dt, A.prev_out + bm);
        return;
    }
    static_assert(EB > 0 && EB < NB, "the d . w_e items and the 2-form positions take blocks of their own");
    const double* E = A.E + int64_t(bm) * 2 * A.n_e;
    const double* H = A.H + int64_t(bm) * 2 * A.n_h;
    const double* we = A.we + int64_t(bm) * A.n_e;
    const double* wh = A.wh + int64_t(bm) * A.n_h;
    const int bx = int(blockIdx.x) - 1;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (bx < EB) {
        // d . w_e, U entries per thread and round, all loads requested before the sums
        const int64_t se = int64_t(EB) * 256;
        for (int64_t ib = int64_t(bx) * 256 + threadIdx.x; ib < A.n_e; ib += U * se) {
            double dv[U], wv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = ib + u * se;
                const bool ok = i < A.n_e;
                const double a = E[A.n_e + (ok ? i : 0)], b = we[ok ? i : 0];
                dv[u] = ok ? a : 0.0;
                wv[u] = ok ? b : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s0 = fma(dv[u], wv[u], s0);
        }
    } else {
        // b . w_h and w_h . D^1 e by positions (z, y, x) of the box that holds
        // the three 2-form components: at each, the components whose dims
        // contain it, (D^1 e)_c = d_{c+1} e_{c+2} - d_{c+2} e_{c+1} from the
        // nine e values around the position, each e value loaded once
        int bz = 0, by = 0, bxn = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            bz = max(bz, A.h_dims[c][0]);
            by = max(by, A.h_dims[c][1]);
            bxn = max(bxn, A.h_dims[c][2]);
        }
        const int npos = bz * by * bxn;
        const int sh = (NB - EB) * 256;
        for (int ip = (bx - EB) * 256 + int(threadIdx.x); ip < npos; ip += sh) {
            int x, y;
            const int row = fast_divmod(ip, bxn, x);
            const int z = fast_divmod(row, by, y);
            double w[3], bb[3];
            bool ok[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int* d = A.h_dims[c];
                ok[c] = z < d[0] && y < d[1] && x < d[2];
                const int64_t j = A.h_comp_off[c] + (ok[c] ? (z * d[1] + y) * d[2] + x : 0);
                w[c] = wh[j];
                bb[c] = H[A.n_h + j];
            }
            // e_a at the position (c) and one step back along a + 1 (m1) and a + 2 (m2)
            double ec[3], m1[3], m2[3];
            e_star<0>(E + A.e_comp_off[0], A.e_dims[0], z, y, x, ec[0], m1[0], m2[0]);
            e_star<1>(E + A.e_comp_off[1], A.e_dims[1], z, y, x, ec[1], m1[1], m2[1]);
            e_star<2>(E + A.e_comp_off[2], A.e_dims[2], z, y, x, ec[2], m1[2], m2[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
                // d_{a1} e_{a2}: e_{a2} back along a1, which is a2 + 2; d_{a2} e_{a1}: e_{a1} back along a2 = a1 + 1
                const double dv = (ec[a2] - m2[a2]) - (ec[a1] - m1[a1]);
                const double wv = ok[c] ? w[c] : 0.0, bv = ok[c] ? bb[c] : 0.0;
                s1 = fma(bv, wv, s1);
                s2 = fma(wv, ok[c] ? dv : 0.0, s2);
            }
        }
    }
    __shared__ double r[3];
    block_sum3<256>(s0, s1, s2, r);
    if (threadIdx.x == 0) {
        double* o = A.partial + (int64_t(bm) * NB + bx) * 3;
        o[0] = r[0];
        o[1] = r[1];
        o[2] = r[2];
    }
}

void launch_energy_dots(const EnergyDotsArgs& a, int batch, hipStream_t s) {
    hipLaunchKernelGGL((energy_dots_kernel<ENERGY_DOT_UNROLL, ENERGY_DOT_EBLOCKS>),
                       dim3(ENERGY_DOT_BLOCKS, batch), dim3(256), 0, s, a);
}

// A dense source pattern times a sampled time series: g(t) by linear
// interpolation of the samples at t0 + k h (zero outside the sampled span),
// then y -= g(t) P over the field.
__global__ void __launch_bounds__(256) pattern_source_kernel(double* y, int64_t y_stride, const double* P,
                                                             int64_t p_stride, int64_t n, const double* series, int m,
                                                             double t0, double h, const double* t_dev, double t_src) {
    const int b = blockIdx.y;
    const double t = (t_dev ? *t_dev : 0.0) + t_src;
    const double u = (t - t0) / h;
    double g = 0.0;
    if (u >= 0.0 && u <= double(m - 1)) {
        const int k = min(int(u), m - 2);
        const double f = u - k;
        g = fma(f, series[k + 1] - series[k], series[k]);
    }
    double* yb = y + int64_t(b) * y_stride;
    const double* pb = P + int64_t(b) * p_stride;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        yb[i] = fma(-g, pb[i], yb[i]);
}

void launch_pattern_source(double* y, int64_t y_stride, const double* P, int64_t p_stride, int64_t n,
                           const double* series, int m, double t0, double h, const double* t_dev, double t_src,
                           int batch, hipStream_t s) {
    const unsigned blocks = unsigned(std::min<int64_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(pattern_source_kernel, dim3(blocks, batch), dim3(256), 0, s, y, y_stride, P, p_stride, n,
                       series, m, t0, h, t_dev, t_src);
}

__global__ void __launch_bounds__(256) energy_final_kernel(const double* partial, int nblocks, double dt,
                                                           double* out, int64_t out_stride) {
    const int b = blockIdx.x;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    constexpr int U = 8;  // partials per thread and round, all requested together
    for (int k0 = 0; k0 < nblocks; k0 += 256 * U) {
        double v[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * 256 + threadIdx.x;
            const double* p = partial + (int64_t(b) * nblocks + (k < nblocks ? k : 0)) * 3;
#pragma unroll
            for (int j = 0; j < 3; ++j) v[u][j] = k < nblocks ? p[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            t0 += v[u][0];
            t1 += v[u][1];
            t2 += v[u][2];
        }
    }
    __shared__ double r[3];
    block_sum3<256>(t0, t1, t2, r);
    __syncthreads();
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
// Adjoint support: transposed curls, probes, per-element permittivity gradient
// ===========================================================================

// out_j = beta out_j + alpha ((D^T y)_j),  (D^T y)_j = d_{j+2}^T y_{j+1} - d_{j+1}^T y_{j+2};
// primal d^T: (d^T u)[c] = u[c] - u[c+1]; dual d~^T: (d~^T u)[j] = u[j-1] - u[j]
__device__ inline double diffT1(const double* u, const int d[3], int primal, int axis, int z, int y, int x) {
    int i[3] = {x, y, z};
    const int n = d[2 - axis];  // length of u along the axis
    auto at = [&](int k) -> double {
        if (k < 0 || k >= n) return 0.0;
        int j[3] = {i[0], i[1], i[2]};
        j[axis] = k;
        return u[(int64_t(j[2]) * d[1] + j[1]) * d[2] + j[0]];
    };
    const int k = i[axis];
    return primal ? at(k) - at(k + 1) : at(k - 1) - at(k);
}

__global__ void curlT_kernel(const CurlArgs A, int64_t n_out) {
    const int b = blockIdx.y;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    int j = 0;
    while (j < 2 && i >= A.out_comp_off[j + 1]) ++j;
    const int64_t li = i - A.out_comp_off[j];
    const int* od = A.out_dims[j];
    const int x = int(li % od[2]), y = int((li / od[2]) % od[1]), z = int(li / (int64_t(od[2]) * od[1]));
    const int c1 = (j + 1) % 3, c2 = (j + 2) % 3;
    const double* in = A.in + int64_t(b) * A.in_stride;
    const double v = diffT1(in + A.in_comp_off[c1], A.in_dims[c1], A.primal, c2, z, y, x) -
                     diffT1(in + A.in_comp_off[c2], A.in_dims[c2], A.primal, c1, z, y, x);
    double* out = A.out + int64_t(b) * A.out_stride;
    out[i] = (A.beta == 0.0 ? 0.0 : A.beta * out[i]) + A.alpha * v;
}

void launch_curlT(const CurlArgs& a, int64_t n_out, int batch, hipStream_t s) {
    dim3 grid(unsigned((n_out + 255) / 256), batch);
    hipLaunchKernelGGL(curlT_kernel, grid, dim3(256), 0, s, a, n_out);
}

// CSR product out[r] = alpha sum_k val[k] x[col[k]] (+ beta out[r]), one thread per row
__global__ void csr_kernel(const int* rowptr, const int* col, const double* val, const double* x, double* out,
                           const int* out_index, int nrows, double alpha, double beta) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) s += val[k] * x[col[k]];
    const int o = out_index ? out_index[r] : r;
    out[o] = (beta == 0.0 ? 0.0 : beta * out[o]) + alpha * s;
}

void launch_csr(const int* rowptr, const int* col, const double* val, const double* x, double* out,
                const int* out_index, int nrows, double alpha, double beta, hipStream_t s) {
    hipLaunchKernelGGL(csr_kernel, dim3((nrows + 255) / 256), dim3(256), 0, s, rowptr, col, val, x, out, out_index,
                       nrows, alpha, beta);
}

// r = obs - data (n values) and the block partial sums of r^2
__global__ void __launch_bounds__(256) residual_kernel(const double* obs, const double* data, double* r, int64_t n,
                                                        double* partial) {
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const double v = obs[i] - data[i];
        r[i] = v;
        s += v * v;
    }
    __shared__ double red[3];
    block_sum3<256>(s, 0.0, 0.0, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

void launch_residual(const double* obs, const double* data, double* r, int64_t n, double* partial, int nblocks,
                     hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(nblocks), dim3(256), 0, s, obs, data, r, n, partial);
}

// dipole terms of the gradient: grad[e0] += coef g(t) (lam . s) / eps_e0, one
// thread, dipoles in a fixed order (after the element kernel, stream-ordered)
__global__ void source_grad_kernel(const double* entries, const double* prof, const int* elem, int n_src,
                                   int entries_per, const double* lam, const int64_t* comp_off, const int* dims,
                                   const double* src_inv_eps, double t, double coef, double* grad) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int k = 0; k < n_src; ++k) {
        if (int(prof[4 * k + 3]) != 0) continue;  // batch member 0 only
        const double dtt = t - prof[4 * k];
        const double gt = prof[4 * k + 2] * exp(-dtt * dtt / (2.0 * prof[4 * k + 1] * prof[4 * k + 1]));
        const double* en = entries + int64_t(k) * entries_per * 5;
        double s = 0.0;
        for (int e = 0; e < entries_per; ++e) {
            const int c = int(en[5 * e]);
            if (c < 0) continue;
            const int iz = int(en[5 * e + 1]), iy = int(en[5 * e + 2]), ix = int(en[5 * e + 3]);
            s += lam[comp_off[c] + (int64_t(iz) * dims[3 * c + 1] + iy) * dims[3 * c + 2] + ix] * en[5 * e + 4];
        }
        grad[elem[k]] += coef * gt * s * src_inv_eps[k];
    }
}

void launch_source_grad(const double* entries, const double* prof, const int* elem, int n_src, int entries_per,
                        const double* lam, const int64_t* comp_off_dev, const int* dims_dev,
                        const double* src_inv_eps, double t, double coef, double* grad, hipStream_t s) {
    hipLaunchKernelGGL(source_grad_kernel, dim3(1), dim3(64), 0, s, entries, prof, elem, n_src, entries_per, lam,
                       comp_off_dev, dims_dev, src_inv_eps, t, coef, grad);
}

// Per-element pairing of two dual 2-forms through the metric,
//   grad_e += coef inv_eps_e^2 sum_{q in e} Lam(q) . G(q) V(q),
// with Lam interpolated from lam and V from the dual curl of the 1-form h.
// Same tiling and sum factorisation as the mass kernel; the element sums are
// reduced over the tile's threads in a fixed order and each tile writes only
// its own elements.
template <int P, int MET>
__global__ void __launch_bounds__(MassCfg<P>::NT) pair_grad_kernel(const PairGradArgs A) {
    constexpr int NQ = P + 1, Q = TILE * NQ, NT = MassCfg<P>::NT;
    using L0 = Lay<P, SP_D, 0>;
    using L1 = Lay<P, SP_D, 1>;
    using L2 = Lay<P, SP_D, 2>;
    using S0 = Lay<P, SP_H, 0>;
    using S1 = Lay<P, SP_H, 1>;
    using S2 = Lay<P, SP_H, 2>;
    constexpr int KMAX = P + 1;
    constexpr int TSL = TILE * NQ * KMAX;
    constexpr int XW = L0::size + L1::size + L2::size;
    constexpr int SW = S0::size + S1::size + S2::size;
    constexpr int BB0 = L0::Wz * Q * L0::Wx, BB1 = L1::Wz * Q * L1::Wx, BB2 = L2::Wz * Q * L2::Wx;
    constexpr int BB = BB0 > BB1 ? (BB0 > BB2 ? BB0 : BB2) : (BB1 > BB2 ? BB1 : BB2);
    constexpr int RED = TILE * Q * Q;
    constexpr int OT = 0, OL = OT + 6 * TSL, OS = OL + XW, OV = OS + SW, OB = OV + XW, OR = OB + BB;
    __shared__ double sm[OR + RED];

    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    const int nt = A.ntile;
    const int tx = tile % nt, ty = (tile / nt) % nt, tz = tile / (nt * nt);
    const int tcoord[3] = {tx, ty, tz};
    const int qy = tid / Q, qx = tid % Q;
    const bool active = tid < Q * Q;

    for (int i = tid; i < 6 * TSL; i += NT) {
        const int a = i / (2 * TSL), slot = (i / TSL) % 2, k = i % TSL;
        const int tag = slot == 0 ? space_tag(SP_D, a, a) : space_tag(SP_D, (a + 1) % 3, a);
        const int K = tag_support(P, tag);
        if (k < TILE * NQ * K) sm[OT + i] = A.tab[A.tab_off[tag] + int64_t(tcoord[a]) * TILE * NQ * K + k];
    }
    load_windows<P, L0, L1, L2, NT>(sm + OL, A.lam, A.lam_comp_off, A.lam_dims, tx, ty, tz, A.n0, A.n1, tid);
    load_windows<P, S0, S1, S2, NT>(sm + OS, A.h, A.h_comp_off, A.h_dims, tx, ty, tz, A.n0, A.n1, tid);
    __syncthreads();
    for (int i = tid; i < XW; i += NT) {
        if (i < L0::size)
            sm[OV + i] = curl_at<P, SP_H, SP_D, 0>(sm + OS, sm + OS + S0::size, sm + OS + S0::size + S1::size, i);
        else if (i < L0::size + L1::size)
            sm[OV + i] = curl_at<P, SP_H, SP_D, 1>(sm + OS, sm + OS + S0::size, sm + OS + S0::size + S1::size,
                                                  i - L0::size);
        else
            sm[OV + i] = curl_at<P, SP_H, SP_D, 2>(sm + OS, sm + OS + S0::size, sm + OS + S0::size + S1::size,
                                                  i - L0::size - L1::size);
    }
    __syncthreads();
    const double* T = sm + OT;
    auto tab = [&](int a, int slot) { return T + (a * 2 + slot) * TSL; };
    double A0[L0::Wz], A1[L1::Wz], A2[L2::Wz], V0[L0::Wz], V1[L1::Wz], V2[L2::Wz];
    contract_xy<P, L0, NQ, Q>(sm + OL, sm + OB, tab(0, 0), tab(1, 1), A0, tid, NT, qy, qx, active);
    contract_xy<P, L1, NQ, Q>(sm + OL + L0::size, sm + OB, tab(0, 1), tab(1, 0), A1, tid, NT, qy, qx, active);
    contract_xy<P, L2, NQ, Q>(sm + OL + L0::size + L1::size, sm + OB, tab(0, 1), tab(1, 1), A2, tid, NT, qy, qx,
                              active);
    contract_xy<P, L0, NQ, Q>(sm + OV, sm + OB, tab(0, 0), tab(1, 1), V0, tid, NT, qy, qx, active);
    contract_xy<P, L1, NQ, Q>(sm + OV + L0::size, sm + OB, tab(0, 1), tab(1, 0), V1, tid, NT, qy, qx, active);
    contract_xy<P, L2, NQ, Q>(sm + OV + L0::size + L1::size, sm + OB, tab(0, 1), tab(1, 1), V2, tid, NT, qy, qx,
                              active);
    double acc[TILE];
#pragma unroll
    for (int le = 0; le < TILE; ++le) acc[le] = 0.0;
    if (active) {
        const double* gm = A.metric + int64_t(tile) * Q * 6 * Q * Q + qy * Q + qx;
        const double* tz0 = tab(2, 1);
        const double* tz2 = tab(2, 0);
        const int64_t npq = int64_t(A.npad) * NQ;
        const int gxq = tx * TILE * NQ + qx, gyq = ty * TILE * NQ + qy;
        double a1 = 0.0, a2 = 0.0, a3 = 0.0, wxy = 0.0;
        if (MET == 1) {
            const double sx = A.axis_tab[gxq], cx = A.axis_tab[npq + gxq], wx = A.axis_tab[2 * npq + gxq];
            const double sy = A.axis_tab[gyq], cy = A.axis_tab[npq + gyq], wy = A.axis_tab[2 * npq + gyq];
            a1 = M_PI * cx * sy;
            a2 = M_PI * sx * cy;
            a3 = M_PI * sx * sy;
            wxy = wx * wy;
        }
        const double amp = A.amp, aa = 3.0 * A.amp * A.amp;
#pragma unroll
        for (int le = 0; le < TILE; ++le) {
#pragma unroll
            for (int iq = 0; iq < NQ; ++iq) {
                const int qz = le * NQ + iq;
                double g[6];
                if (MET == 1) {
                    const int gzq = tz * TILE * NQ + qz;
                    const double sz = A.axis_tab[gzq], cz = A.axis_tab[npq + gzq], wz = A.axis_tab[2 * npq + gzq];
                    const double p1 = a1 * sz, p2 = a2 * sz, p3 = a3 * cz;
                    const double f = wxy * wz * recip_nr(1.0 + amp * (p1 + p2 + p3));
                    g[0] = f * (1.0 + 2.0 * amp * p1 + aa * p1 * p1);
                    g[1] = f * (1.0 + 2.0 * amp * p2 + aa * p2 * p2);
                    g[2] = f * (1.0 + 2.0 * amp * p3 + aa * p3 * p3);
                    g[3] = f * (amp * (p1 + p2) + aa * p1 * p2);
                    g[4] = f * (amp * (p1 + p3) + aa * p1 * p3);
                    g[5] = f * (amp * (p2 + p3) + aa * p2 * p3);
                } else {
#pragma unroll
                    for (int k = 0; k < 6; ++k) g[k] = gm[int64_t(qz) * 6 * Q * Q + k * Q * Q];
                }
                const double* t0 = tz0 + (le * NQ + iq) * L0::Kz;
                const double* t2 = tz2 + (le * NQ + iq) * L2::Kz;
                double l0 = 0.0, l1 = 0.0, l2 = 0.0, v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
                for (int j = 0; j < L0::Kz; ++j) {
                    l0 += t0[j] * A0[le + j];
                    v0 += t0[j] * V0[le + j];
                }
#pragma unroll
                for (int j = 0; j < L1::Kz; ++j) {
                    l1 += t0[j] * A1[le + j];
                    v1 += t0[j] * V1[le + j];
                }
#pragma unroll
                for (int j = 0; j < L2::Kz; ++j) {
                    l2 += t2[j] * A2[le + j];
                    v2 += t2[j] * V2[le + j];
                }
                acc[le] += l0 * (g[0] * v0 + g[3] * v1 + g[4] * v2) + l1 * (g[3] * v0 + g[1] * v1 + g[5] * v2) +
                           l2 * (g[4] * v0 + g[5] * v1 + g[2] * v2);
            }
        }
#pragma unroll
        for (int le = 0; le < TILE; ++le) sm[OR + (le * Q + qy) * Q + qx] = acc[le];
    }
    __syncthreads();
    if (tid < TILE * TILE * TILE) {
        const int lex = tid % TILE, ley = (tid / TILE) % TILE, lez = tid / (TILE * TILE);
        const int ex = tx * TILE + lex, ey = ty * TILE + ley, ez = tz * TILE + lez;
        if (ex < A.N && ey < A.N && ez < A.N) {
            double s = 0.0;
            for (int iy = 0; iy < NQ; ++iy)
                for (int ix = 0; ix < NQ; ++ix) s += sm[OR + (lez * Q + ley * NQ + iy) * Q + lex * NQ + ix];
            const double ie = A.inv_eps[(int64_t(ez) * A.npad + ey) * A.npad + ex];
            A.grad[(int64_t(ez) * A.N + ey) * A.N + ex] += A.coef * ie * ie * s;
        }
    }
}

void launch_pair_grad(int p, const PairGradArgs& a, hipStream_t s) {
    const int nt3 = a.ntile * a.ntile * a.ntile;
#define LP(PP)                                                                                            \
    if (p == PP) {                                                                                        \
        if (a.metric_mode == 1)                                                                           \
            hipLaunchKernelGGL((pair_grad_kernel<PP, 1>), dim3(nt3), dim3(MassCfg<PP>::NT), 0, s, a);     \
        else                                                                                              \
            hipLaunchKernelGGL((pair_grad_kernel<PP, 0>), dim3(nt3), dim3(MassCfg<PP>::NT), 0, s, a);     \
        return;                                                                                           \
    }
    LP(2) LP(3) LP(4)
#undef LP
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

__global__ void advance_time_kernel(double* t, double dt) {
    if (threadIdx.x == 0) t[0] += dt;
}

void launch_advance_time(double* t, double dt, hipStream_t s) {
    hipLaunchKernelGGL(advance_time_kernel, dim3(1), dim3(64), 0, s, t, dt);
}

__global__ void fill_kernel(double* x, int64_t n, double v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

void launch_fill(double* x, int64_t n, double v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(fill_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, x, n, v);
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

// r.r and r.z in one pass: per-block partials [block][2], then one
// fixed-order final sum writing the two results to separate scalars.
__global__ void __launch_bounds__(256) dot2_kernel(const double* r, const double* z, int64_t n, double* partial) {
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const double a = r[i];
        s0 += a * a;
        s1 += a * z[i];
    }
    __shared__ double red[3];
    block_sum3<256>(s0, s1, 0.0, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0];
        partial[2 * blockIdx.x + 1] = red[1];
    }
}

__global__ void __launch_bounds__(256) sum2_final_kernel(const double* partial, int nblocks, double* out0,
                                                         double* out1) {
    double s0 = 0.0, s1 = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += 256) {
        s0 += partial[2 * k];
        s1 += partial[2 * k + 1];
    }
    __shared__ double red[3];
    block_sum3<256>(s0, s1, 0.0, red);
    if (threadIdx.x == 0) {
        out0[0] = red[0];
        out1[0] = red[1];
    }
}

void launch_dot2(const double* r, const double* z, int64_t n, double* partial, int nblocks, double* out0,
                 double* out1, hipStream_t s) {
    hipLaunchKernelGGL(dot2_kernel, dim3(nblocks), dim3(256), 0, s, r, z, n, partial);
    hipLaunchKernelGGL(sum2_final_kernel, dim3(1), dim3(256), 0, s, partial, nblocks, out0, out1);
}

// CG updates with the step scalars addressed explicitly (alternating slots
// for r.z, so no copies between iterations):
//   phase 0: x += a p, r -= a Ap   (a = num / den)
//   phase 1: p = z + b p           (b = num / den)
__global__ void cg2_kernel(double* x, double* r, double* pdir, const double* Ap, const double* z, int64_t n,
                           const double* num, const double* den, int phase) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // a zero denominator (a zero right-hand side, or a residual already zero
    // in a fixed-count solve) makes the step a no-op
    const double c = den[0] != 0.0 ? num[0] / den[0] : 0.0;
    if (phase == 0) {
        x[i] += c * pdir[i];
        r[i] -= c * Ap[i];
    } else {
        pdir[i] = z[i] + c * pdir[i];
    }
}

void launch_cg2(double* x, double* r, double* pdir, const double* Ap, const double* z, int64_t n, const double* num,
                const double* den, int phase, hipStream_t s) {
    hipLaunchKernelGGL(cg2_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, x, r, pdir, Ap, z, n, num, den,
                       phase);
}

void launch_cg_update(double* x, double* r, double* pdir, const double* Ap, const double* z, int64_t n,
                      const double* scal, int phase, hipStream_t s) {
    hipLaunchKernelGGL(cg_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, x, r, pdir, Ap, z, n, scal,
                       phase);
}

}  // namespace kmx
