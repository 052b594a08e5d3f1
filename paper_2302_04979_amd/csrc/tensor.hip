// Spaces with a degree, a knot vector and an element count per direction
// (Section 4.1: with p_i and Xi_i per direction the pairing blocks keep the
// Kronecker form of eqs. (4.2)/(4.3), each 1D factor built from the bases of
// its own direction, and each solve stays one banded 1D solve per axis,
// eqs. (4.4)-(4.5)).  The spaces are the tensor products of the univariate
// spaces of Section 2.3, now per direction; the curls are the same index
// differences (Section 2.4); the 2-form masses (Section 3.4) integrate over
// per-direction Gauss rules with p_i + 1 points per element.
//
// Device layout: fields as in the single-degree spaces (three components one
// after the other, x fastest inside); the 1D basis tables per direction and
// tag, element-major [e][q][k] and zero past the last element up to a whole
// tile; per direction and Gauss point (sin(pi x), cos(pi x), w), from which
// the mass kernel forms the metric factor w_q DF^T DF / det DF of the map at
// every point (the identity and the deformed cube are the maps taken; points
// of padded elements have w = 0); the mass apply writes, per tile and component, the
// tile's window of basis functions (TT + K - 1 per direction) with the x rows
// of the tiles side by side ([tz][ty][wz][wy][tx][wx]), and the gather sums
// for each output the (at most eight) tile windows that hold it in a fixed
// order.  The pairing solves run the banded line kernels of the single-degree
// spaces, with the factors of every direction padded to the half bandwidth of
// the largest degree (the padding holds zeros, so the substitutions are
// unchanged).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "kmx_internal.hpp"
#include "setup.hpp"

namespace kmx {

kmx_status report_error(kmx_status st, const std::string& msg);  // api.hip
std::vector<double> pairing_inverse(const std::vector<double>& A, int n);  // api.hip

namespace {

constexpr int TP_MAX = 4;                            // largest degree per direction
constexpr int TK = TP_MAX + 1;                       // functions per element and direction (at most)
constexpr int TLINE_MAX = 76;                        // longest 1D space the line kernels hold

constexpr int TT = 4;                                // elements per tile edge of the mass apply

// Arguments of the tiled mass apply (one workgroup per tile of TT^3 elements).
struct TMassArgs {
    const double* x;
    int64_t x_stride;
    double* patch;
    int64_t patch_stride;        // per member
    const double* tab;
    int64_t tab_off[3][4];       // [direction][tag] -> [nt TT elements][nq][K], zero past N
    int nt[3];                   // tiles per direction
    int N[3];
    int64_t comp_off[3];
    int dims[3][3];              // [c][z, y, x]
    int64_t pcomp_off[3];        // patch region of each component
    const double* geo;           // per direction: [nt TT][nq][3] = sin(pi x), cos(pi x), w
    int64_t geo_off[3];
    double amp;                  // map amplitude a (0: the identity)
    const double* inv_gamma;     // per element (x fastest)
    // with the curl fused: x is the 1-form (layout src_*), the windows are
    // formed from its differences; track (optional) += talpha (the curl) on
    // the 2-form entries the tile owns
    int64_t src_comp_off[3];
    int src_dims[3][3];
    double* track;
    int64_t track_stride;
    double talpha;
};

struct TGatherArgs {
    const double* patch;
    int64_t patch_stride;
    double* out;
    int64_t out_stride;
    int nt[3];
    int64_t comp_off[3];
    int dims[3][3];
    int64_t pcomp_off[3];
};

// Block index -> work item so that each of the 8 XCDs (which take blocks
// round robin) walks one contiguous range: neighbouring tiles, which share
// window entries and patch lines, then meet in the same L2.
__device__ inline int t_xcd_order(int block, int nblocks) {
    constexpr int XCD = 8;
    const int per = nblocks / XCD;
    return block < per * XCD ? (block % XCD) * per + block / XCD : block;
}

// One difference of the incidence matrices (Section 2.4) along `axis` at
// (z, y, x): primal v[k] - v[k-1], dual v[k+1] - v[k], zero outside 0..n-1.
__device__ inline double t_diff(const double* u, const int d[3], int primal, int axis, int z, int y, int x) {
    const int n = d[2 - axis];
    const int k = axis == 0 ? x : (axis == 1 ? y : z);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? d[2] : int64_t(d[1]) * d[2]);
    const int64_t base = (int64_t(z) * d[1] + y) * d[2] + x;
    const int hi = primal ? k : k + 1, lo = hi - 1;
    const double a = (hi >= 0 && hi < n) ? u[base + (hi - k) * stride] : 0.0;
    const double b = (lo >= 0 && lo < n) ? u[base + (lo - k) * stride] : 0.0;
    return a - b;
}

// 1/d by the hardware's reciprocal estimate and two Newton-Raphson steps
// r <- r + r (1 - d r), each of which squares the relative error.
__device__ inline double t_recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// Window of component C of a 2-form space over one tile, per direction: the
// functions nonzero on one element (K), the tile window W = TT + K - 1 and the
// offset of local index 0 in the global numbering.
template <int PX, int PY, int PZ, int SPACE, int C>
struct TWin {
    static constexpr int Kx = tag_support(PX, space_tag(SPACE, C, 0));
    static constexpr int Ky = tag_support(PY, space_tag(SPACE, C, 1));
    static constexpr int Kz = tag_support(PZ, space_tag(SPACE, C, 2));
    static constexpr int ox = tag_offset(space_tag(SPACE, C, 0));
    static constexpr int oy = tag_offset(space_tag(SPACE, C, 1));
    static constexpr int oz = tag_offset(space_tag(SPACE, C, 2));
    static constexpr int Wx = TT + Kx - 1, Wy = TT + Ky - 1, Wz = TT + Kz - 1;
    static constexpr int size = Wx * Wy * Wz;
    // the table slot (0: the tag along the component, 1: across) per direction
    static constexpr int sx = C == 0 ? 0 : 1, sy = C == 1 ? 0 : 1, sz = C == 2 ? 0 : 1;
};

// Patch layout of one component: [tz][ty][wz][wy][tx][wx], the x rows of the
// tiles along x side by side (a gather wave reading a row of outputs touches
// contiguous memory).
template <class Wn>
__device__ inline int64_t t_patch_at(const int nt[3], int tx, int ty, int tz, int wx, int wy, int wz) {
    return ((((int64_t(tz) * nt[1] + ty) * Wn::Wz + wz) * Wn::Wy + wy) * nt[0] + tx) * Wn::Wx + wx;
}

constexpr int t_max3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }

// threads of a tiled mass workgroup: one per (qy, qx) column of the tile
constexpr int tt_threads(int px, int py) { return ((TT * (px + 1) * TT * (py + 1) + 63) / 64) * 64; }

template <int PX, int PY, int PZ>
struct TTile {
    static constexpr int NQX = PX + 1, NQY = PY + 1, NQZ = PZ + 1;
    static constexpr int QX = TT * NQX, QY = TT * NQY, QZ = TT * NQZ;
    static constexpr int NT = tt_threads(PX, PY);
    static constexpr int QM = t_max3(QX, QY, QZ);
};

// Interpolation of component C along x and y: the tile window into LDS, the x
// pass into LDS, the y pass into the thread's register column A[wz] (the
// window's z planes at the thread's (qy, qx)).
template <int PX, int PY, int PZ, int SPACE, bool CURL, int C, int WZM>
__device__ inline void tt_forward_xy(const TMassArgs& A, const double* x, double* track,
                                     double (*tab)[2][TTile<PX, PY, PZ>::QM * TK], double* X, double* AX,
                                     const int t3[3], int tid, int qy, int qx, bool active, double (&col)[WZM]) {
    using Wn = TWin<PX, PY, PZ, SPACE, C>;
    using T = TTile<PX, PY, PZ>;
    const int nx = A.dims[C][2], ny = A.dims[C][1], nz = A.dims[C][0];
    const int gx0 = t3[0] * TT + Wn::ox, gy0 = t3[1] * TT + Wn::oy, gz0 = t3[2] * TT + Wn::oz;
    const double* xc = x + A.comp_off[C];
    constexpr int A1 = (C + 1) % 3, A2 = (C + 2) % 3;
    for (int i = tid; i < Wn::size; i += T::NT) {
        const int wx = i % Wn::Wx, wy = (i / Wn::Wx) % Wn::Wy, wz = i / (Wn::Wx * Wn::Wy);
        const int gx = gx0 + wx, gy = gy0 + wy, gz = gz0 + wz;
        const bool ok = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
        double v = 0.0;
        if (CURL) {
            // component C of the curl of the 1-form at this entry
            if (ok) {
                constexpr int primal = SPACE == SP_B ? 1 : 0;
                v = t_diff(x + A.src_comp_off[A2], A.src_dims[A2], primal, A1, gz, gy, gx) -
                    t_diff(x + A.src_comp_off[A1], A.src_dims[A1], primal, A2, gz, gy, gx);
                // the tracked 2-form's update on the entries this tile owns
                // (local index below TT, or any in the last tile of a direction)
                const bool own = (wx < TT || t3[0] == A.nt[0] - 1) && (wy < TT || t3[1] == A.nt[1] - 1) &&
                                 (wz < TT || t3[2] == A.nt[2] - 1);
                if (track && own) {
                    double* t = track + A.comp_off[C] + (int64_t(gz) * ny + gy) * nx + gx;
                    *t = *t + A.talpha * v;
                }
            }
        } else {
            v = ok ? xc[(int64_t(gz) * ny + gy) * nx + gx] : 0.0;
        }
        X[i] = v;
    }
    __syncthreads();
    const double* tx = tab[0][Wn::sx];
    for (int i = tid; i < Wn::Wz * Wn::Wy * T::QX; i += T::NT) {
        const int q = i % T::QX, r = i / T::QX;  // r = wz * Wy + wy
        const int ex = q / T::NQX;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < Wn::Kx; ++k) s += tx[q * TK + k] * X[r * Wn::Wx + ex + k];
        AX[i] = s;
    }
    __syncthreads();
    if (active) {
        const double* ty = tab[1][Wn::sy];
        const int ey = qy / T::NQY;
#pragma unroll
        for (int wz = 0; wz < Wn::Wz; ++wz) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < Wn::Ky; ++k) s += ty[qy * TK + k] * AX[(wz * Wn::Wy + ey + k) * T::QX + qx];
            col[wz] = s;
        }
    }
    __syncthreads();  // X and AX are reused by the next component
}

// Integration of component C along x and y: the thread's column R[wz] into
// LDS; a thread per (wz, qy) row integrates it along x against the x table
// (each Gauss point qx feeds the K_x functions of its element, no masked
// terms) into XI[wz][wx][qy]; a thread per (wz, wx) column integrates that
// along y likewise and writes the column of the tile's patch.
template <int PX, int PY, int PZ, int SPACE, int C, int WZM>
__device__ inline void tt_backward_xy(const TMassArgs& A, double* patch, double (*tab)[2][TTile<PX, PY, PZ>::QM * TK],
                                      double* RB, double* XI, const int t3[3], int tid, int qy, int qx, bool active,
                                      const double (&col)[WZM]) {
    using Wn = TWin<PX, PY, PZ, SPACE, C>;
    using T = TTile<PX, PY, PZ>;
    constexpr int XP = T::QY + 1;  // odd pitch of the XI columns
    constexpr int RP = T::QX + 1;  // odd pitch of the RB rows (the x integration reads one row per lane)
    static_assert(Wn::Wz * T::QY <= T::NT && Wn::Wz * Wn::Wx <= T::NT, "a thread per row and per column");
    if (active) {
#pragma unroll
        for (int wz = 0; wz < Wn::Wz; ++wz) RB[(wz * T::QY + qy) * RP + qx] = col[wz];
    }
    __syncthreads();
    if (tid < Wn::Wz * T::QY) {
        const double* tx = tab[0][Wn::sx];
        const int wz = tid / T::QY, y = tid - wz * T::QY;
        const double* row = RB + (wz * T::QY + y) * RP;
        double r[T::QX];
#pragma unroll
        for (int q = 0; q < T::QX; ++q) r[q] = row[q];
        double c[Wn::Wx];
#pragma unroll
        for (int w = 0; w < Wn::Wx; ++w) c[w] = 0.0;
#pragma unroll
        for (int q = 0; q < T::QX; ++q) {
            const int le = q / T::NQX;
#pragma unroll
            for (int k = 0; k < Wn::Kx; ++k) c[le + k] = fma(tx[q * TK + k], r[q], c[le + k]);
        }
#pragma unroll
        for (int w = 0; w < Wn::Wx; ++w) XI[(wz * Wn::Wx + w) * XP + y] = c[w];
    }
    __syncthreads();
    if (tid < Wn::Wz * Wn::Wx) {
        const double* ty = tab[1][Wn::sy];
        const int wz = tid / Wn::Wx, wx = tid - wz * Wn::Wx;
        const double* cl = XI + tid * XP;
        double cq[T::QY];
#pragma unroll
        for (int q = 0; q < T::QY; ++q) cq[q] = cl[q];
        double o[Wn::Wy];
#pragma unroll
        for (int w = 0; w < Wn::Wy; ++w) o[w] = 0.0;
#pragma unroll
        for (int q = 0; q < T::QY; ++q) {
            const int le = q / T::NQY;
#pragma unroll
            for (int k = 0; k < Wn::Ky; ++k) o[le + k] = fma(ty[q * TK + k], cq[q], o[le + k]);
        }
        double* pc = patch + A.pcomp_off[C];
#pragma unroll
        for (int w = 0; w < Wn::Wy; ++w) pc[t_patch_at<Wn>(A.nt, t3[0], t3[1], t3[2], wx, w, wz)] = o[w];
    }
    __syncthreads();  // RB and XI are reused by the next component
}

// One workgroup per tile of TT^3 elements, one thread per (qy, qx) Gauss
// column of the tile: the x and y contractions of each component through LDS
// into register columns, then a walk over the tile's Gauss planes (z
// interpolation, the metric factor formed per point, 1/gamma of the point's
// element, the z integration back into register columns), then the y and x
// integrations into the tile's patch.  Specialised on the three degrees.
template <int PX, int PY, int PZ, int SPACE, bool CURL>
__global__ void __launch_bounds__(tt_threads(PX, PY)) ttile_mass_kernel(const TMassArgs A) {
    using T = TTile<PX, PY, PZ>;
    using W0 = TWin<PX, PY, PZ, SPACE, 0>;
    using W1 = TWin<PX, PY, PZ, SPACE, 1>;
    using W2 = TWin<PX, PY, PZ, SPACE, 2>;
    constexpr int WSZ = t_max3(W0::size, W1::size, W2::size);
    constexpr int WZM = t_max3(W0::Wz, W1::Wz, W2::Wz);
    // x passes (forward) and the x integrals XI[wz][wx][qy] (backward, pitch QY + 1)
    constexpr int AXF = t_max3(W0::Wz * W0::Wy, W1::Wz * W1::Wy, W2::Wz * W2::Wy) * T::QX;
    constexpr int AXB = t_max3(W0::Wz * W0::Wx, W1::Wz * W1::Wx, W2::Wz * W2::Wx) * (T::QY + 1);
    constexpr int AXN = AXF > AXB ? AXF : AXB;
    constexpr int RBN = WZM * T::QY * (T::QX + 1);
    __shared__ double tab[3][2][T::QM * TK];
    __shared__ double X[WSZ];
    __shared__ double AX[AXN];   // x pass (forward), x integrals (backward)
    __shared__ double RB[RBN];
    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    const int ntile = A.nt[0] * A.nt[1] * A.nt[2];
    const int tile = t_xcd_order(blockIdx.x, ntile);
    const int t3[3] = {tile % A.nt[0], (tile / A.nt[0]) % A.nt[1], tile / (A.nt[0] * A.nt[1])};
    const int qy = tid / T::QX, qx = tid % T::QX;
    const bool active = tid < T::QX * T::QY;
    const double* x = A.x + int64_t(b) * A.x_stride;
    double* track = A.track ? A.track + int64_t(b) * A.track_stride : nullptr;

    // the tile's 1D tables, both tags of the space per direction
    {
        constexpr int NQ[3] = {T::NQX, T::NQY, T::NQZ};
        constexpr int PD[3] = {PX, PY, PZ};
        for (int i = tid; i < 3 * 2 * T::QM * TK; i += T::NT) {
            const int a = i / (2 * T::QM * TK), s = (i / (T::QM * TK)) % 2, q = (i / TK) % T::QM, k = i % TK;
            const int tag = space_tag(SPACE, s == 0 ? a : (a + 1) % 3, a);
            const int K = tag_support(PD[a], tag);
            double v = 0.0;
            if (q < TT * NQ[a] && k < K) v = A.tab[A.tab_off[a][tag] + (int64_t(t3[a]) * TT * NQ[a] + q) * K + k];
            tab[a][s][q * TK + k] = v;
        }
    }
    // the map values of the tile's Gauss points, per direction
    __shared__ double geo[3][T::QM][3];
    {
        constexpr int NQ[3] = {T::NQX, T::NQY, T::NQZ};
        for (int i = tid; i < 3 * T::QM * 3; i += T::NT) {
            const int a = i / (T::QM * 3), q = (i / 3) % T::QM, k = i % 3;
            geo[a][q][k] = q < TT * NQ[a] ? A.geo[A.geo_off[a] + (int64_t(t3[a]) * TT * NQ[a] + q) * 3 + k] : 0.0;
        }
    }
    // 1/gamma of the elements of this thread's column (padded elements: their
    // weights are zero)
    double ig[TT];
    {
        const int ex = min(t3[0] * TT + qx / T::NQX, A.N[0] - 1), ey = min(t3[1] * TT + qy / T::NQY, A.N[1] - 1);
#pragma unroll
        for (int ez = 0; ez < TT; ++ez) {
            const int gz = min(t3[2] * TT + ez, A.N[2] - 1);
            ig[ez] = active ? A.inv_gamma[(int64_t(gz) * A.N[1] + ey) * A.N[0] + ex] : 0.0;
        }
    }
    __syncthreads();

    double a0[WZM], a1[WZM], a2[WZM];
#pragma unroll
    for (int k = 0; k < WZM; ++k) a0[k] = a1[k] = a2[k] = 0.0;
    tt_forward_xy<PX, PY, PZ, SPACE, CURL, 0, WZM>(A, x, track, tab, X, AX, t3, tid, qy, qx, active, a0);
    tt_forward_xy<PX, PY, PZ, SPACE, CURL, 1, WZM>(A, x, track, tab, X, AX, t3, tid, qy, qx, active, a1);
    tt_forward_xy<PX, PY, PZ, SPACE, CURL, 2, WZM>(A, x, track, tab, X, AX, t3, tid, qy, qx, active, a2);

    // the walk over the tile's Gauss planes
    double r0[WZM], r1[WZM], r2[WZM];
#pragma unroll
    for (int k = 0; k < WZM; ++k) r0[k] = r1[k] = r2[k] = 0.0;
    if (active) {
        const double* tz0 = tab[2][W0::sz];
        const double* tz1 = tab[2][W1::sz];
        const double* tz2 = tab[2][W2::sz];
        // G = w DF^T DF / det DF of F(x) = x + a s(x) (1, 1, 1),
        // s = sin(pi x) sin(pi y) sin(pi z): with q = a grad s, DF = I + 1 q^T,
        // det DF = 1 + q . 1 and DF^T DF = I + q 1^T + 1 q^T + 3 q q^T, so
        // G v = f (v + (S + 3 Q) q + Q 1) with f = w / det DF, S = sum v and
        // Q = q . v: a rank-2 update of the identity, f scaled by 1/gamma
        const double am = A.amp;
        const double sx = geo[0][qx][0], cx = geo[0][qx][1], wx = geo[0][qx][2];
        const double sy = geo[1][qy][0], cy = geo[1][qy][1], wy = geo[1][qy][2];
        const double pcs = am * M_PI * cx * sy, psc = am * M_PI * sx * cy, pss = am * M_PI * sx * sy;
        const double wxy = wx * wy;
#pragma unroll
        for (int qz = 0; qz < T::QZ; ++qz) {
            const int ez = qz / T::NQZ;
            const double sz = geo[2][qz][0], cz = geo[2][qz][1], wz = geo[2][qz][2];
            const double q1 = pcs * sz, q2 = psc * sz, q3 = pss * cz;
            const double sf = (ig[ez] * (wxy * wz)) * t_recip(1.0 + (q1 + q2 + q3));
            double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
            for (int k = 0; k < W0::Kz; ++k) v0 += tz0[qz * TK + k] * a0[ez + k];
#pragma unroll
            for (int k = 0; k < W1::Kz; ++k) v1 += tz1[qz * TK + k] * a1[ez + k];
#pragma unroll
            for (int k = 0; k < W2::Kz; ++k) v2 += tz2[qz * TK + k] * a2[ez + k];
            const double Qv = fma(q1, v0, fma(q2, v1, q3 * v2));
            const double cq = sf * fma(3.0, Qv, v0 + v1 + v2), bq = sf * Qv;
            const double u0 = fma(sf, v0, fma(cq, q1, bq));
            const double u1 = fma(sf, v1, fma(cq, q2, bq));
            const double u2 = fma(sf, v2, fma(cq, q3, bq));
#pragma unroll
            for (int k = 0; k < W0::Kz; ++k) r0[ez + k] += tz0[qz * TK + k] * u0;
#pragma unroll
            for (int k = 0; k < W1::Kz; ++k) r1[ez + k] += tz1[qz * TK + k] * u1;
#pragma unroll
            for (int k = 0; k < W2::Kz; ++k) r2[ez + k] += tz2[qz * TK + k] * u2;
        }
    }
    double* patch = A.patch + int64_t(b) * A.patch_stride;
    tt_backward_xy<PX, PY, PZ, SPACE, 0, WZM>(A, patch, tab, RB, AX, t3, tid, qy, qx, active, r0);
    tt_backward_xy<PX, PY, PZ, SPACE, 1, WZM>(A, patch, tab, RB, AX, t3, tid, qy, qx, active, r1);
    tt_backward_xy<PX, PY, PZ, SPACE, 2, WZM>(A, patch, tab, RB, AX, t3, tid, qy, qx, active, r2);
}

// out_i = sum of the patch entries of the (at most eight) tiles whose window
// holds function i, by increasing z, y, x tile index.
template <int PX, int PY, int PZ, int SPACE, int C>
__device__ inline double tt_gather_one(const TGatherArgs& A, const double* patch, int gx, int gy, int gz) {
    using Wn = TWin<PX, PY, PZ, SPACE, C>;
    const int r[3] = {gx - Wn::ox, gy - Wn::oy, gz - Wn::oz};
    const int W[3] = {Wn::Wx, Wn::Wy, Wn::Wz};
    int t[3][2], w[3][2];
    bool v[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int h = r[a] / TT;
        h = h > A.nt[a] - 1 ? A.nt[a] - 1 : h;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int c = h - 1 + d;
            v[a][d] = c >= 0 && r[a] - c * TT < W[a];
            t[a][d] = v[a][d] ? c : h;
            w[a][d] = v[a][d] ? r[a] - c * TT : 0;
        }
    }
    const double* pc = patch + A.pcomp_off[C];
    double s = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                // only the lanes whose candidate covers the entry read it
                double val = 0.0;
                if (v[2][dz] && v[1][dy] && v[0][dx])
                    val = pc[t_patch_at<Wn>(A.nt, t[0][dx], t[1][dy], t[2][dz], w[0][dx], w[1][dy], w[2][dz])];
                s += val;
            }
    return s;
}

template <int PX, int PY, int PZ, int SPACE>
__global__ void __launch_bounds__(256) ttile_gather_kernel(const TGatherArgs A, int64_t n) {
    const int b = blockIdx.y;
    const int64_t i = int64_t(t_xcd_order(blockIdx.x, gridDim.x)) * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = i >= A.comp_off[2] ? 2 : (i >= A.comp_off[1] ? 1 : 0);
    const int64_t li = i - A.comp_off[c];
    const int nx = A.dims[c][2], ny = A.dims[c][1];
    const int gx = int(li % nx), gy = int((li / nx) % ny), gz = int(li / (int64_t(nx) * ny));
    const double* patch = A.patch + int64_t(b) * A.patch_stride;
    double s;
    if (c == 0) s = tt_gather_one<PX, PY, PZ, SPACE, 0>(A, patch, gx, gy, gz);
    else if (c == 1) s = tt_gather_one<PX, PY, PZ, SPACE, 1>(A, patch, gx, gy, gz);
    else s = tt_gather_one<PX, PY, PZ, SPACE, 2>(A, patch, gx, gy, gz);
    A.out[int64_t(b) * A.out_stride + i] = s;
}

// out = D^1 in (primal) or D~^1 in (dual), component c = d_{c+1} in_{c+2} -
// d_{c+2} in_{c+1}; with `track`, also track += talpha (the same curl): the
// tracked 2-form's update from the differences already formed.
__global__ void __launch_bounds__(256) t_curl_kernel(const CurlArgs A, double* track, int64_t track_stride,
                                                     double talpha, int64_t n_out) {
    const int b = blockIdx.y;
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n_out) return;
    const int c = i >= A.out_comp_off[2] ? 2 : (i >= A.out_comp_off[1] ? 1 : 0);
    const int64_t li = i - A.out_comp_off[c];
    const int* od = A.out_dims[c];
    const int x = int(li % od[2]), y = int((li / od[2]) % od[1]), z = int(li / (int64_t(od[2]) * od[1]));
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    const double* in = A.in + int64_t(b) * A.in_stride;
    const double v = t_diff(in + A.in_comp_off[a2], A.in_dims[a2], A.primal, a1, z, y, x) -
                     t_diff(in + A.in_comp_off[a1], A.in_dims[a1], A.primal, a2, z, y, x);
    A.out[int64_t(b) * A.out_stride + i] = v;
    if (track) {
        double* t = track + int64_t(b) * track_stride + i;
        *t = *t + talpha * v;
    }
}

template <int PX, int PY, int PZ>
void t_launch_p(const TMassArgs& m, const TGatherArgs& g, int64_t n, int batch, hipStream_t s, int space, bool curl) {
    const int ntile = m.nt[0] * m.nt[1] * m.nt[2];
    const dim3 gm(unsigned(ntile), batch), gg(unsigned((n + 255) / 256), batch);
    const dim3 bm(TTile<PX, PY, PZ>::NT);
    if (space == SP_B) {
        if (curl) hipLaunchKernelGGL((ttile_mass_kernel<PX, PY, PZ, SP_B, true>), gm, bm, 0, s, m);
        else hipLaunchKernelGGL((ttile_mass_kernel<PX, PY, PZ, SP_B, false>), gm, bm, 0, s, m);
        hipLaunchKernelGGL((ttile_gather_kernel<PX, PY, PZ, SP_B>), gg, dim3(256), 0, s, g, n);
    } else {
        if (curl) hipLaunchKernelGGL((ttile_mass_kernel<PX, PY, PZ, SP_D, true>), gm, bm, 0, s, m);
        else hipLaunchKernelGGL((ttile_mass_kernel<PX, PY, PZ, SP_D, false>), gm, bm, 0, s, m);
        hipLaunchKernelGGL((ttile_gather_kernel<PX, PY, PZ, SP_D>), gg, dim3(256), 0, s, g, n);
    }
}

// the mass kernel and the gather for the space's degrees (2..4 each)
void t_launch_mass(const int p[3], const TMassArgs& m, const TGatherArgs& g, int64_t n, int batch, hipStream_t s,
                   int space, bool curl) {
    const int code = (p[0] - 2) * 9 + (p[1] - 2) * 3 + (p[2] - 2);
#define TL(PX, PY, PZ)                                                       \
    case (PX - 2) * 9 + (PY - 2) * 3 + (PZ - 2):                             \
        t_launch_p<PX, PY, PZ>(m, g, n, batch, s, space, curl);              \
        return;
#define TL3(PX, PY) TL(PX, PY, 2) TL(PX, PY, 3) TL(PX, PY, 4)
    switch (code) {
        TL3(2, 2) TL3(2, 3) TL3(2, 4)
        TL3(3, 2) TL3(3, 3) TL3(3, 4)
        TL3(4, 2) TL3(4, 3) TL3(4, 4)
        default: return;
    }
#undef TL3
#undef TL
}

// ---------------------------------------------------------------------------
// host set-up
// ---------------------------------------------------------------------------
struct TAxis {
    int p = 0, N = 0, nq = 0, n0 = 0, n1 = 0;
    std::vector<double> t;                   // p-open knot vector
    std::vector<double> xq, wq;              // Gauss points and weights, element by element
    std::vector<double> tab[4];              // [nt TT][nq][K(tag)], zero past the N elements
    std::vector<double> G, M;                // dense 1D pairing matrices
};

// Values of the functions of `tag` nonzero on element e at x (knot vector t of
// degree p; trimmed vectors Xi', Xi'' for the lower degrees).
void t_eval(const TAxis& ax, int tag, int e, double x, double* vals) {
    const int p = ax.p;
    const std::vector<double>& t = ax.t;
    if (tag == PV) {
        nonzero_bsplines(t, p + e, p, x, vals);  // functions e .. e + p of the whole basis
        for (int j = 0; j <= p; ++j) {
            const int gidx = e + j - 1;  // index without the first boundary function
            if (gidx < 0 || gidx >= ax.n0) vals[j] = 0.0;
        }
    } else if (tag == PD || tag == DV) {
        const std::vector<double> t1(t.begin() + 1, t.end() - 1);
        nonzero_bsplines(t1, p - 1 + e, p - 1, x, vals);  // e .. e + p - 1
        if (tag == PD)
            for (int j = 0; j < p; ++j) vals[j] *= p / (t1[e + j + p] - t1[e + j]);  // unit integrals
    } else {
        const std::vector<double> t2(t.begin() + 2, t.end() - 2);
        nonzero_bsplines(t2, p - 2 + e, p - 2, x, vals);  // e .. e + p - 2
        for (int j = 0; j < p - 1; ++j) vals[j] *= (p - 1) / (t2[e + j + p - 1] - t2[e + j]);
    }
}

void t_build_axis(TAxis& ax, int p, int N, const double* breaks) {
    ax.p = p;
    ax.N = N;
    ax.nq = p + 1;
    ax.n0 = N + p - 2;
    ax.n1 = N + p - 1;
    std::vector<double> nodes(N + 1);
    for (int k = 0; k <= N; ++k) nodes[k] = breaks && k > 0 && k < N ? breaks[k - 1] : double(k) / N;
    nodes[0] = 0.0;
    nodes[N] = 1.0;
    for (int k = 0; k < N; ++k)
        if (!(nodes[k + 1] > nodes[k])) throw std::invalid_argument("breakpoints must increase inside (0, 1)");
    ax.t.assign(p + 1, 0.0);
    for (int k = 1; k < N; ++k) ax.t.push_back(nodes[k]);
    for (int k = 0; k <= p; ++k) ax.t.push_back(1.0);
    std::vector<double> g, gw;
    gauss_legendre(ax.nq, g, gw);
    ax.xq.resize(size_t(N) * ax.nq);
    ax.wq.resize(size_t(N) * ax.nq);
    for (int e = 0; e < N; ++e)
        for (int q = 0; q < ax.nq; ++q) {
            const double h = nodes[e + 1] - nodes[e];
            ax.xq[e * ax.nq + q] = nodes[e] + 0.5 * (g[q] + 1.0) * h;
            ax.wq[e * ax.nq + q] = 0.5 * gw[q] * h;
        }
    for (int tag = 0; tag < 4; ++tag) {
        const int K = tag_support(p, tag);
        const int npad = ((N + TT - 1) / TT) * TT;
        ax.tab[tag].assign(size_t(npad) * ax.nq * K, 0.0);
        for (int e = 0; e < N; ++e)
            for (int q = 0; q < ax.nq; ++q) t_eval(ax, tag, e, ax.xq[e * ax.nq + q], &ax.tab[tag][(e * ax.nq + q) * K]);
    }
    // G^ = int Dd^T Pv (n0 x n0), M^ = int Dv^T Pd (n1 x n1), Section 4.1
    const int n0 = ax.n0, n1 = ax.n1;
    ax.G.assign(size_t(n0) * n0, 0.0);
    ax.M.assign(size_t(n1) * n1, 0.0);
    const int Kpv = p + 1, Kpd = p, Kdv = p, Kdd = p - 1;
    for (int e = 0; e < N; ++e)
        for (int q = 0; q < ax.nq; ++q) {
            const double w = ax.wq[e * ax.nq + q];
            const double* dd = &ax.tab[DD][(e * ax.nq + q) * Kdd];
            const double* pv = &ax.tab[PV][(e * ax.nq + q) * Kpv];
            const double* dv = &ax.tab[DV][(e * ax.nq + q) * Kdv];
            const double* pd = &ax.tab[PD][(e * ax.nq + q) * Kpd];
            for (int i = 0; i < Kdd; ++i)
                for (int j = 0; j < Kpv; ++j) {
                    const int r = e + i, cidx = e + j - 1;
                    if (cidx >= 0 && cidx < n0) ax.G[r * n0 + cidx] += w * dd[i] * pv[j];
                }
            for (int i = 0; i < Kdv; ++i)
                for (int j = 0; j < Kpd; ++j) ax.M[(e + i) * n1 + (e + j)] += w * dv[i] * pd[j];
        }
}

std::vector<double> transpose_sq(const std::vector<double>& A, int n) {
    std::vector<double> T(A.size());
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) T[j * n + i] = A[i * n + j];
    return T;
}

}  // namespace
}  // namespace kmx

using namespace kmx;

struct kmx_tspace {
    int p[3] = {0, 0, 0}, N[3] = {0, 0, 0};
    int pmax = 0, max_batch = 1;
    int map_kind = 0;
    double amplitude = 0.0;
    int64_t n_e = 0, n_h = 0, nfield = 0, nelem = 0;
    TAxis ax[3];
    int dims[4][3][3];          // per space (SP_E..SP_D): [c][z, y, x]
    int64_t comp_off[4][3];
    int nt[3] = {0, 0, 0};      // tiles of TT elements per direction
    int64_t pcomp_off[4][3];    // patch regions of the components (tile windows)
    int64_t psize[4] = {0, 0, 0, 0};  // patch doubles of one field, all components
    int64_t psize_max = 0;
    int64_t tab_off[3][4];
    int64_t fac_off[3][4];      // [direction][F_G, F_M, F_GT, F_MT]
    // dense FP64 inverses of the 1D factors in the matrix cores' operand
    // order (lines of at most DENSE_NMAX entries): the solves' dense form
    double* d_frag = nullptr;
    int64_t frag_off[3][4];     // [direction][F_G, F_M, F_GT, F_MT]
    int dense_ok = 0;           // the dense inverses exist
    int dense = 0;              // the solves use them (kmx_tspace_set_solver)
    double* d_tab = nullptr;
    double* d_fac = nullptr;
    double* d_geo = nullptr;
    int64_t geo_off[3] = {0, 0, 0};
    double* d_inv_eps = nullptr;
    double* d_inv_mu = nullptr;
    double* d_patch = nullptr;
    double* d_u = nullptr;      // curl output
    double* d_y = nullptr;      // gathered mass output
    double* d_t = nullptr;      // between the xy and z passes of a solve
};

namespace {

kmx_status t_fail(kmx_status st, const std::string& msg) { return report_error(st, msg); }

#define T_TRY(expr)                                                                          \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return t_fail(KMX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define T_CHECK_LAUNCH()                                                                     \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess) return t_fail(KMX_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

kmx_status t_upload(double** dst, const std::vector<double>& v) {
    if (hipMalloc(dst, std::max<size_t>(v.size(), 1) * sizeof(double)) != hipSuccess)
        return t_fail(KMX_E_OOM, "device allocation failed");
    if (!v.empty()) T_TRY(hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    return KMX_OK;
}

// det DF > 0 at every Gauss point of the map (F(x) = x + a s(x) (1, 1, 1):
// det DF = 1 + a (s_x + s_y + s_z))
kmx_status t_check_map(const kmx_tspace* ts) {
    if (ts->map_kind != 1) return KMX_OK;
    const TAxis &X = ts->ax[0], &Y = ts->ax[1], &Z = ts->ax[2];
    const double a = ts->amplitude;
    for (int kz = 0; kz < Z.N * Z.nq; ++kz)
        for (int ky = 0; ky < Y.N * Y.nq; ++ky)
            for (int kx = 0; kx < X.N * X.nq; ++kx) {
                const double sx = std::sin(M_PI * X.xq[kx]), sy = std::sin(M_PI * Y.xq[ky]),
                             sz = std::sin(M_PI * Z.xq[kz]);
                const double cx = std::cos(M_PI * X.xq[kx]), cy = std::cos(M_PI * Y.xq[ky]),
                             cz = std::cos(M_PI * Z.xq[kz]);
                const double det = 1.0 + a * M_PI * (cx * sy * sz + sx * cy * sz + sx * sy * cz);
                if (!(det > 0.0) || !std::isfinite(det)) return t_fail(KMX_E_GEOMETRY, "det DF <= 0 at a quadrature point");
            }
    return KMX_OK;
}

// 1/gamma per element (host values gamma, x fastest; NULL = 1)
kmx_status t_upload_inverse(kmx_tspace* ts, const double* g, double* dst) {
    std::vector<double> v(size_t(ts->nelem), 1.0);
    if (g)
        for (int64_t k = 0; k < ts->nelem; ++k) {
            if (!(g[k] > 0.0) || !std::isfinite(g[k])) return t_fail(KMX_E_MATERIAL, "eps and mu must be positive");
            v[k] = 1.0 / g[k];
        }
    T_TRY(hipMemcpy(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    return KMX_OK;
}

// which_K1 = 1: K1 (blocks of eq. (4.2)); 0: K~1 (eq. (4.3)).  The factor of
// direction a for component c.
int t_pair_kind(int which_K1, int transpose, int c, int a) {
    if (which_K1) return transpose ? (a == c ? F_MT : F_GT) : (a == c ? F_M : F_G);
    return transpose ? (a == c ? F_G : F_M) : (a == c ? F_GT : F_MT);
}

// x = K^{-1} y (solve = 1) or K y (solve = 2), then out = (acc ? out : 0) + alpha x;
// y and out hold `batch` fields of the layout of K's rows (= columns).
void t_solve(kmx_tspace* ts, int which_K1, int transpose, const double* y, int64_t y_stride, double* out,
             int64_t out_stride, double alpha, int accumulate, int solve, int batch, hipStream_t s) {
    const int layout = which_K1 ? SP_D : SP_B;
    if (solve == 1 && ts->dense) {
        // B_y Y B_x^T per z plane, then B_z along z, with the dense inverses
        DenseArgs d{};
        for (int c = 0; c < 3; ++c) {
            d.comp_off[c] = ts->comp_off[layout][c];
            for (int k = 0; k < 3; ++k) d.dims[c][k] = ts->dims[layout][c][k];
            for (int ax = 0; ax < 3; ++ax) d.frag_off[c][ax] = ts->frag_off[ax][t_pair_kind(which_K1, transpose, c, ax)];
        }
        d.frag = ts->d_frag;
        d.in = y;
        d.in_stride = y_stride;
        d.out = ts->d_t;
        d.out_stride = ts->nfield;
        launch_dense_xy(d, batch, s);
        d.in = ts->d_t;
        d.in_stride = ts->nfield;
        d.out = out;
        d.out_stride = out_stride;
        d.alpha = alpha;
        d.accumulate = accumulate;
        launch_dense_z(d, batch, s);
        return;
    }
    XYArgs a{};
    a.in = y;
    a.in_stride = y_stride;
    a.out = ts->d_t;
    a.out_stride = ts->nfield;
    for (int c = 0; c < 3; ++c) {
        a.comp_off[c] = ts->comp_off[layout][c];
        for (int k = 0; k < 3; ++k) a.dims[c][k] = ts->dims[layout][c][k];
    }
    // six factor sets per call: direction a's "along" (slot 2a) and "across" (2a + 1)
    a.fac = ts->d_fac;
    for (int ax = 0; ax < 3; ++ax) {
        a.fac_off[2 * ax] = ts->fac_off[ax][t_pair_kind(which_K1, transpose, ax, ax)];
        a.fac_off[2 * ax + 1] = ts->fac_off[ax][t_pair_kind(which_K1, transpose, (ax + 1) % 3, ax)];
    }
    for (int c = 0; c < 3; ++c)
        for (int ax = 0; ax < 3; ++ax) a.fac_id[c][ax] = 2 * ax + (ax == c ? 0 : 1);
    a.n_src = 0;
    a.solve = solve;
    launch_xy(ts->pmax, a, batch, s);
    ZArgs z{};
    z.in = ts->d_t;
    z.in_stride = ts->nfield;
    z.out = out;
    z.out_stride = out_stride;
    for (int c = 0; c < 3; ++c) {
        z.comp_off[c] = a.comp_off[c];
        for (int k = 0; k < 3; ++k) z.dims[c][k] = a.dims[c][k];
        z.fac_id[c] = a.fac_id[c][2];
    }
    z.fac = ts->d_fac;
    for (int k = 0; k < 8; ++k) z.fac_off[k] = a.fac_off[k];
    z.alpha = alpha;
    z.accumulate = accumulate;
    z.solve = solve;
    launch_z(ts->pmax, z, batch, s);
}

// y = M x (space SP_B: M^2_{1/mu}; SP_D: M~^2_{1/eps}) for `batch` fields;
// with `curl`, y = M D x for the 1-form x (D^1 for B, D~^1 for D) and, when
// track is given, track += talpha D x
void t_mass(kmx_tspace* ts, int space, const double* x, int64_t x_stride, double* y, int64_t y_stride, int batch,
            hipStream_t s, bool curl = false, double* track = nullptr, int64_t track_stride = 0, double talpha = 0.0) {
    TMassArgs m{};
    if (curl) {
        const int src = space == SP_B ? SP_E : SP_H;
        for (int c = 0; c < 3; ++c) {
            m.src_comp_off[c] = ts->comp_off[src][c];
            for (int k = 0; k < 3; ++k) m.src_dims[c][k] = ts->dims[src][c][k];
        }
        m.track = track;
        m.track_stride = track_stride;
        m.talpha = talpha;
    }
    m.x = x;
    m.x_stride = x_stride;
    m.patch = ts->d_patch;
    m.patch_stride = ts->psize_max;
    m.tab = ts->d_tab;
    for (int a = 0; a < 3; ++a) {
        for (int t = 0; t < 4; ++t) m.tab_off[a][t] = ts->tab_off[a][t];
        m.nt[a] = ts->nt[a];
        m.N[a] = ts->N[a];
    }
    for (int c = 0; c < 3; ++c) {
        m.comp_off[c] = ts->comp_off[space][c];
        m.pcomp_off[c] = ts->pcomp_off[space][c];
        for (int k = 0; k < 3; ++k) m.dims[c][k] = ts->dims[space][c][k];
    }
    m.geo = ts->d_geo;
    for (int a = 0; a < 3; ++a) m.geo_off[a] = ts->geo_off[a];
    m.amp = ts->map_kind == 1 ? ts->amplitude : 0.0;
    m.inv_gamma = space == SP_B ? ts->d_inv_mu : ts->d_inv_eps;
    TGatherArgs g{};
    g.patch = ts->d_patch;
    g.patch_stride = m.patch_stride;
    g.out = y;
    g.out_stride = y_stride;
    for (int a = 0; a < 3; ++a) g.nt[a] = ts->nt[a];
    for (int c = 0; c < 3; ++c) {
        g.comp_off[c] = m.comp_off[c];
        g.pcomp_off[c] = m.pcomp_off[c];
        for (int k = 0; k < 3; ++k) g.dims[c][k] = m.dims[c][k];
    }
    const int64_t n = space == SP_B ? ts->n_h : ts->n_e;
    t_launch_mass(ts->p, m, g, n, batch, s, space, curl);
}

// out = D^1 in (primal) or D~^1 in (dual); track (optional) += talpha (the curl)
void t_curl(kmx_tspace* ts, int primal, const double* in, int64_t in_stride, double* out, int64_t out_stride,
            double* track, int64_t track_stride, double talpha, int batch, hipStream_t s) {
    CurlArgs a{};
    a.in = in;
    a.in_stride = in_stride;
    a.out = out;
    a.out_stride = out_stride;
    a.alpha = 1.0;
    a.beta = 0.0;
    a.primal = primal;
    const int si = primal ? SP_E : SP_H, so = primal ? SP_B : SP_D;
    for (int c = 0; c < 3; ++c) {
        a.in_comp_off[c] = ts->comp_off[si][c];
        a.out_comp_off[c] = ts->comp_off[so][c];
        for (int k = 0; k < 3; ++k) {
            a.in_dims[c][k] = ts->dims[si][c][k];
            a.out_dims[c][k] = ts->dims[so][c][k];
        }
    }
    const int64_t n = primal ? ts->n_h : ts->n_e;
    hipLaunchKernelGGL(t_curl_kernel, dim3(unsigned((n + 255) / 256), batch), dim3(256), 0, s, a, track, track_stride,
                       talpha, n);
}

}  // namespace

extern "C" {

kmx_status kmx_create_tspace(const int* p, const int* n_elem, const double* breaks_x, const double* breaks_y,
                             const double* breaks_z, const kmx_map* map, int max_batch, kmx_tspace** out) {
    if (!out || !p || !n_elem) return t_fail(KMX_E_ARG, "NULL argument");
    *out = nullptr;
    if (max_batch < 1) return t_fail(KMX_E_ARG, "max_batch < 1");
    const int kind = map ? map->kind : 0;
    if (kind != 0 && kind != 1) return t_fail(KMX_E_ARG, "per-direction spaces take map kinds 0 and 1");
    for (int a = 0; a < 3; ++a) {
        if (p[a] < 2 || p[a] > TP_MAX) return t_fail(KMX_E_ARG, "degree per direction must be 2..4");
        if (n_elem[a] < 1 || n_elem[a] + p[a] - 1 > TLINE_MAX)
            return t_fail(KMX_E_ARG, "elements per direction: 1 .. 77 - p");
    }
    kmx_tspace* ts = new kmx_tspace();
    const double* br[3] = {breaks_x, breaks_y, breaks_z};
    try {
        for (int a = 0; a < 3; ++a) {
            ts->p[a] = p[a];
            ts->N[a] = n_elem[a];
            t_build_axis(ts->ax[a], p[a], n_elem[a], br[a]);
        }
    } catch (const std::exception& ex) {
        delete ts;
        return t_fail(KMX_E_ARG, ex.what());
    }
    ts->pmax = std::max(p[0], std::max(p[1], p[2]));
    ts->max_batch = max_batch;
    ts->map_kind = kind;
    ts->amplitude = map ? map->amplitude : 0.0;
    ts->nelem = int64_t(n_elem[0]) * n_elem[1] * n_elem[2];
    // per space: component dims (z, y, x), offsets, and patch windows
    for (int a = 0; a < 3; ++a) ts->nt[a] = (n_elem[a] + TT - 1) / TT;
    for (int sp = 0; sp < 4; ++sp) {
        int64_t off = 0, poff = 0;
        for (int c = 0; c < 3; ++c) {
            ts->comp_off[sp][c] = off;
            ts->pcomp_off[sp][c] = poff;
            int64_t n = 1, w = 1;
            for (int a = 0; a < 3; ++a) {
                const int tag = space_tag(sp, c, a);
                const int d = (tag == PV || tag == DD) ? ts->ax[a].n0 : ts->ax[a].n1;
                ts->dims[sp][c][2 - a] = d;
                n *= d;
                w *= int64_t(ts->nt[a]) * (TT + tag_support(p[a], tag) - 1);  // tile windows along a
            }
            off += n;
            poff += w;
        }
        ts->psize[sp] = poff;
        if (sp == SP_E) ts->n_e = off;
        if (sp == SP_H) ts->n_h = off;
    }
    ts->psize_max = std::max(ts->psize[SP_B], ts->psize[SP_D]);
    ts->nfield = std::max(ts->n_e, ts->n_h);
    kmx_status st;
    std::vector<double> tabs;
    for (int a = 0; a < 3; ++a)
        for (int t = 0; t < 4; ++t) {
            ts->tab_off[a][t] = int64_t(tabs.size());
            tabs.insert(tabs.end(), ts->ax[a].tab[t].begin(), ts->ax[a].tab[t].end());
        }
    if ((st = t_upload(&ts->d_tab, tabs)) != KMX_OK) { kmx_destroy_tspace(ts); return st; }
    // banded LU factors of G^, M^ and their transposes per direction, all with
    // the half bandwidth of the largest degree
    std::vector<double> facs;
    try {
        for (int a = 0; a < 3; ++a) {
            const TAxis& A = ts->ax[a];
            const BandLU sets[4] = {band_lu(A.G, A.n0, ts->pmax - 1), band_lu(A.M, A.n1, ts->pmax - 1),
                                    band_lu(transpose_sq(A.G, A.n0), A.n0, ts->pmax - 1),
                                    band_lu(transpose_sq(A.M, A.n1), A.n1, ts->pmax - 1)};
            for (int k = 0; k < 4; ++k) {
                ts->fac_off[a][k] = int64_t(facs.size());
                facs.insert(facs.end(), sets[k].L.begin(), sets[k].L.end());
                facs.insert(facs.end(), sets[k].U.begin(), sets[k].U.end());
                facs.insert(facs.end(), sets[k].dinv.begin(), sets[k].dinv.end());
                facs.insert(facs.end(), sets[k].band.begin(), sets[k].band.end());
            }
        }
    } catch (const std::exception& ex) {
        kmx_destroy_tspace(ts);
        return t_fail(KMX_E_ARG, std::string("pairing factors: ") + ex.what());
    }
    if ((st = t_upload(&ts->d_fac, facs)) != KMX_OK) { kmx_destroy_tspace(ts); return st; }
    {
        // the dense form of the solves when every line fits the dense kernels
        // and their planes fit the LDS
        int nmax = 0;
        for (int a = 0; a < 3; ++a) nmax = std::max(nmax, ts->ax[a].n1);
        int dev = 0, max_lds = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            kmx_destroy_tspace(ts);
            return t_fail(KMX_E_DEVICE, "device attributes");
        }
        const size_t shm = std::max(dense_lds_bytes(ts->dims[SP_B]), dense_lds_bytes(ts->dims[SP_D]));
        if (nmax <= DENSE_NMAX && shm <= size_t(max_lds)) {
            std::vector<double> frag;
            try {
                for (int a = 0; a < 3; ++a)
                    for (int k = 0; k < 4; ++k) {
                        const TAxis& A = ts->ax[a];
                        const int n = (k == F_G || k == F_GT) ? A.n0 : A.n1;
                        const std::vector<double> Ai = pairing_inverse((k == F_G || k == F_GT) ? A.G : A.M, n);
                        std::vector<double> B(size_t(n) * n);
                        const bool tr = k == F_GT || k == F_MT;
                        for (int i = 0; i < n; ++i)
                            for (int j = 0; j < n; ++j) B[size_t(i) * n + j] = tr ? Ai[size_t(j) * n + i] : Ai[size_t(i) * n + j];
                        ts->frag_off[a][k] = int64_t(frag.size());
                        frag.resize(frag.size() + size_t(dense_frag_doubles(n)));
                        dense_fragments(B.data(), n, frag.data() + ts->frag_off[a][k]);
                    }
            } catch (const std::exception& ex) {
                kmx_destroy_tspace(ts);
                return t_fail(KMX_E_ARG, std::string("pairing inverses: ") + ex.what());
            }
            if ((st = t_upload(&ts->d_frag, frag)) != KMX_OK) { kmx_destroy_tspace(ts); return st; }
            if (dense_prepare(shm) != hipSuccess) {
                kmx_destroy_tspace(ts);
                return t_fail(KMX_E_DEVICE, "dense solve kernels: LDS grant failed");
            }
            ts->dense_ok = 1;
            ts->dense = 1;
        }
    }
    {
        if ((st = t_check_map(ts)) != KMX_OK) { kmx_destroy_tspace(ts); return st; }
        // per direction (sin(pi x), cos(pi x), w) at the Gauss points, zero
        // past the last element up to a whole tile
        std::vector<double> geo;
        for (int a = 0; a < 3; ++a) {
            ts->geo_off[a] = int64_t(geo.size());
            const TAxis& A = ts->ax[a];
            const int npad = ts->nt[a] * TT;
            for (int k = 0; k < npad * A.nq; ++k) {
                const bool in = k < A.N * A.nq;
                geo.push_back(in ? std::sin(M_PI * A.xq[k]) : 0.0);
                geo.push_back(in ? std::cos(M_PI * A.xq[k]) : 0.0);
                geo.push_back(in ? A.wq[k] : 0.0);
            }
        }
        if ((st = t_upload(&ts->d_geo, geo)) != KMX_OK) { kmx_destroy_tspace(ts); return st; }
    }
    const size_t nf = size_t(ts->nfield) * max_batch;
    if (hipMalloc(&ts->d_inv_eps, size_t(ts->nelem) * sizeof(double)) != hipSuccess ||
        hipMalloc(&ts->d_inv_mu, size_t(ts->nelem) * sizeof(double)) != hipSuccess ||
        hipMalloc(&ts->d_patch, size_t(ts->psize_max) * max_batch * sizeof(double)) != hipSuccess ||
        hipMalloc(&ts->d_u, nf * sizeof(double)) != hipSuccess ||
        hipMalloc(&ts->d_y, nf * sizeof(double)) != hipSuccess ||
        hipMalloc(&ts->d_t, nf * sizeof(double)) != hipSuccess) {
        kmx_destroy_tspace(ts);
        return t_fail(KMX_E_OOM, "device allocation failed (scratch)");
    }
    if ((st = t_upload_inverse(ts, nullptr, ts->d_inv_eps)) != KMX_OK ||
        (st = t_upload_inverse(ts, nullptr, ts->d_inv_mu)) != KMX_OK) {
        kmx_destroy_tspace(ts);
        return st;
    }
    *out = ts;
    return KMX_OK;
}

void kmx_destroy_tspace(kmx_tspace* ts) {
    if (!ts) return;
    double* bufs[] = {ts->d_tab, ts->d_fac, ts->d_frag, ts->d_geo, ts->d_inv_eps, ts->d_inv_mu,
                      ts->d_patch, ts->d_u, ts->d_y, ts->d_t};
    for (double* b : bufs)
        if (b) (void)hipFree(b);
    delete ts;
}

kmx_status kmx_tspace_sizes(const kmx_tspace* ts, int64_t* n_e, int64_t* n_h) {
    if (!ts) return t_fail(KMX_E_ARG, "space is NULL");
    if (n_e) *n_e = ts->n_e;
    if (n_h) *n_h = ts->n_h;
    return KMX_OK;
}

kmx_status kmx_tspace_set_materials(kmx_tspace* ts, const double* eps_elem, const double* mu_elem) {
    if (!ts) return t_fail(KMX_E_ARG, "space is NULL");
    // validate both before changing either
    for (const double* g : {eps_elem, mu_elem})
        if (g)
            for (int64_t k = 0; k < ts->nelem; ++k)
                if (!(g[k] > 0.0) || !std::isfinite(g[k])) return t_fail(KMX_E_MATERIAL, "eps and mu must be positive");
    kmx_status st;
    if ((st = t_upload_inverse(ts, eps_elem, ts->d_inv_eps)) != KMX_OK) return st;
    return t_upload_inverse(ts, mu_elem, ts->d_inv_mu);
}

kmx_status kmx_tspace_set_solver(kmx_tspace* ts, int dense) {
    if (!ts || (dense != 0 && dense != 1)) return t_fail(KMX_E_ARG, "bad argument");
    if (dense && !ts->dense_ok) return t_fail(KMX_E_STATE, "no dense factors for this space (a line above 80 entries)");
    ts->dense = dense;
    return KMX_OK;
}

kmx_status kmx_tspace_op_curl(kmx_tspace* ts, int which, const double* x, double* y, void* stream) {
    if (!ts || !x || !y || (which != 0 && which != 1)) return t_fail(KMX_E_ARG, "bad argument");
    const int primal = which == 0;
    t_curl(ts, primal, x, primal ? ts->n_e : ts->n_h, y, primal ? ts->n_h : ts->n_e, nullptr, 0, 0.0, 1,
           static_cast<hipStream_t>(stream));
    T_CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_tspace_op_mass(kmx_tspace* ts, int which, const double* x, double* y, void* stream) {
    if (!ts || !x || !y || (which != 0 && which != 1)) return t_fail(KMX_E_ARG, "bad argument");
    const int space = which == 0 ? SP_B : SP_D;
    const int64_t n = which == 0 ? ts->n_h : ts->n_e;
    t_mass(ts, space, x, n, y, n, 1, static_cast<hipStream_t>(stream));
    T_CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_tspace_op_solve(kmx_tspace* ts, int which, int transpose, const double* y, double* x, void* stream) {
    if (!ts || !x || !y || (which != 0 && which != 1)) return t_fail(KMX_E_ARG, "bad argument");
    const int64_t n = which ? ts->n_e : ts->n_h;
    t_solve(ts, which, transpose ? 1 : 0, y, n, x, n, 1.0, 0, 1, 1, static_cast<hipStream_t>(stream));
    T_CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_tspace_op_pairing(kmx_tspace* ts, int which, const double* x, double* y, void* stream) {
    if (!ts || !x || !y || (which != 0 && which != 1)) return t_fail(KMX_E_ARG, "bad argument");
    const int64_t n = which ? ts->n_e : ts->n_h;
    t_solve(ts, which, 0, x, n, y, n, 1.0, 0, 2, 1, static_cast<hipStream_t>(stream));
    T_CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_tspace_step(kmx_tspace* ts, double* E, double* H, double dt, int nsteps, int batch, int flags,
                           void* stream) {
    if (!ts || !E || !H) return t_fail(KMX_E_ARG, "NULL argument");
    if (batch < 1 || batch > ts->max_batch) return t_fail(KMX_E_ARG, "batch out of range");
    if (nsteps < 0) return t_fail(KMX_E_ARG, "nsteps < 0");
    if (!std::isfinite(dt)) return t_fail(KMX_E_ARG, "dt not finite");
    const int track = flags & KMX_TRACK_DB;
    const int64_t es = ts->n_e * (1 + track), hs = ts->n_h * (1 + track);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int n = 0; n < nsteps; ++n) {
        // h -= dt K~1^{-1} M D^1 e   (b -= dt D^1 e)
        t_mass(ts, SP_B, E, es, ts->d_y, ts->nfield, batch, s, true, track ? H + ts->n_h : nullptr, hs, -dt);
        t_solve(ts, 0, 0, ts->d_y, ts->nfield, H, hs, -dt, 1, 1, batch, s);
        // e += dt K1^{-1} M~ D~^1 h   (d += dt D~^1 h)
        t_mass(ts, SP_D, H, hs, ts->d_y, ts->nfield, batch, s, true, track ? E + ts->n_e : nullptr, es, dt);
        t_solve(ts, 1, 0, ts->d_y, ts->nfield, E, es, dt, 1, 1, batch, s);
    }
    T_CHECK_LAUNCH();
    return KMX_OK;
}

}  // extern "C"
