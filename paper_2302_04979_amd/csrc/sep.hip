// Persistent leapfrog for separable spaces: identity map and uniform eps, mu.
//
// With F = id the 2-form metric is the identity, so the Hodge matrices of
// Section 3.4 are Kronecker products of 1D Gram matrices (scaled by 1/mu and
// 1/eps), exactly as the pairings K1, K~1 are Kronecker products of the 1D
// G^, M^ (eqs. (4.2)-(4.3)).  One half step of component c is then
//     curl -> three banded Gram products -> (source) -> three banded solves,
// a chain of mode-n products along x, y and z of one component tensor.  At
// the sizes where the tensor fits one workgroup's LDS (p = 3: N <= 25), the
// whole chain runs there and each batch member is owned by one workgroup for
// all of its steps: one launch advances every member by nsteps, with only
// workgroup barriers (members never exchange data).
//
// Each mode product is a per-thread pass over the lines of that axis: the
// line is loaded from LDS into registers, the banded Gram product and the
// banded LU substitution run in registers, and the line is written back.
#include "kernels.hpp"

namespace kmx {

namespace {

// The two values whose difference is (d v)[k] = v[k] - v[k-1] (primal, zero
// outside) or v[k+1] - v[k] (dual) of component array u (dims [z, y, x])
// along `axis`, at the output position (z, y, x).
__device__ inline void diff_pair(const double* u, const int d[3], int primal, int axis, int z, int y, int x,
                                 double& hi, double& lo) {
    const int sy = d[2], sz = d[1] * d[2];
    const int idx = z * sz + y * sy + x;
    const int st = axis == 0 ? 1 : (axis == 1 ? sy : sz);
    const int k = axis == 0 ? x : (axis == 1 ? y : z);
    if (primal) {
        hi = k < d[2 - axis] ? u[idx] : 0.0;
        lo = k >= 1 ? u[idx - st] : 0.0;
    } else {
        hi = u[idx + st];
        lo = u[idx];
    }
}

// Position (x, y, z) of the thread's m-th entry tid + m * nthr of a [z][y][x]
// grid, advanced by carries instead of integer divisions (which the GPU
// emulates in software) per entry.
struct GridWalk {
    int x, y, z, dx, dy, dz, nx, ny;
    __device__ GridWalk(int tid, int nthr, int nx_, int ny_) : nx(nx_), ny(ny_) {
        x = tid % nx;
        y = (tid / nx) % ny;
        z = tid / (nx * ny);
        dx = nthr % nx;
        dy = (nthr / nx) % ny;
        dz = nthr / (nx * ny);
    }
    __device__ void next() {
        x += dx;
        const int cx = x >= nx;
        x -= cx ? nx : 0;
        y += dy + cx;
        const int cy = y >= ny;
        y -= cy ? ny : 0;
        z += dz + cy;
    }
};

// Curl of component c of the 1-form `src` (primal or dual) into the LDS
// tensor of the 2-form grid od, with the optional tracking update
// trk += talpha * curl.  U entries per thread are loaded before any is used,
// so that each thread keeps several global loads in flight.
template <int U>
__device__ inline void curl_to_lds(double* buf, const double* src, const int64_t soff[3], const int sdims[3][3],
                                   int primal, int c, const int od[3], double* trk, double talpha, int tid,
                                   int nthr) {
    const int nz = od[0], ny = od[1], nx = od[2], pitch = nx | 1;
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    GridWalk g(tid, nthr, nx, ny);
    for (int i0 = tid; i0 < nz * ny * nx; i0 += U * nthr) {
        double p0[U], p1[U], q0[U], q1[U], tv[U];
        int li[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            li[u] = -1;
            p0[u] = p1[u] = q0[u] = q1[u] = tv[u] = 0.0;
            if (g.z < nz) {
                li[u] = (g.z * ny + g.y) * pitch + g.x;
                diff_pair(src + soff[a2], sdims[a2], primal, a1, g.z, g.y, g.x, p0[u], p1[u]);
                diff_pair(src + soff[a1], sdims[a1], primal, a2, g.z, g.y, g.x, q0[u], q1[u]);
                if (trk) tv[u] = trk[i0 + u * nthr];
            }
            g.next();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (li[u] >= 0) {
                const double v = (p0[u] - p1[u]) - (q0[u] - q1[u]);
                buf[li[u]] = v;
                if (trk) trk[i0 + u * nthr] = tv[u] + talpha * v;
            }
        }
    }
}

// dst += alpha * (LDS tensor), U entries per thread in flight.
template <int U>
__device__ inline void update_from_lds(double* dst, const double* buf, const int od[3], double alpha, int tid,
                                       int nthr) {
    const int nx = od[2], pitch = nx | 1, rows = od[0] * od[1], cnt = rows * nx;
    GridWalk g(tid, nthr, nx, rows);  // (x, row) walk; z stays 0
    for (int i0 = tid; i0 < cnt; i0 += U * nthr) {
        double v[U];
        int li[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nthr;
            li[u] = g.z == 0 ? g.y * pitch + g.x : -1;
            v[u] = (i < cnt) ? dst[i] : 0.0;
            g.next();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nthr;
            if (i < cnt) dst[i] = v[u] + alpha * buf[li[u]];
        }
    }
}

// y = scale * (band x) in registers; band rows hold 2P+1 entries of half
// width P (zeros outside the matrix); entries i >= n stay zero.
template <int P, int LMAX>
__device__ inline void gram_regs(double (&r)[LMAX], int n, const double* __restrict__ band, double scale) {
    constexpr int B = 2 * P + 1;
    double win[P];  // the P original entries before i
#pragma unroll
    for (int m = 0; m < P; ++m) win[m] = 0.0;
#pragma unroll
    for (int i = 0; i < LMAX; ++i) {
        double s = 0.0;
        if (i < n) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int j = i - P + k;
                const double v = k < P ? win[k] : (j < LMAX ? r[j] : 0.0);
                s += band[i * B + k] * v;
            }
        }
#pragma unroll
        for (int m = 0; m + 1 < P; ++m) win[m] = win[m + 1];
        win[P - 1] = r[i];
        r[i] = s * scale;
    }
}

// x = (LU)^{-1} r in registers, banded factors of half width W = P-1.
template <int P, int LMAX>
__device__ inline void lu_regs(double (&r)[LMAX], int n, const double* __restrict__ L, const double* __restrict__ U,
                               const double* __restrict__ dinv) {
    constexpr int W = P - 1;
#pragma unroll
    for (int i = 1; i < LMAX; ++i) {
        if (i < n) {
            double s = r[i];
#pragma unroll
            for (int m = 0; m < W; ++m)
                if (i - 1 - m >= 0) s -= L[i * W + m] * r[i - 1 - m];
            r[i] = s;
        }
    }
#pragma unroll
    for (int i = LMAX - 1; i >= 0; --i) {
        if (i < n) {
            double s = r[i];
#pragma unroll
            for (int m = 0; m < W; ++m)
                if (i + 1 + m < LMAX) s -= U[i * W + m] * r[i + 1 + m];
            r[i] = s * dinv[i];
        }
    }
}

enum { OP_GRAM = 1, OP_SOLVE = 2 };
constexpr int CH = 4;  // entries per chunk of global loads (divides every LMAX)

// Line view of the LDS tensor (dims [z, y, x], row pitch `pitch`): line l of
// `axis` starts at base and steps by stride.
__device__ inline void line_of(int axis, int l, const int d[3], int pitch, int& base, int& stride) {
    const int ny = d[1], nx = d[2];
    if (axis == 0) {          // l = z*ny + y
        base = l * pitch;
        stride = 1;
    } else if (axis == 1) {   // l = z*nx + x
        base = (l / nx) * ny * pitch + (l % nx);
        stride = pitch;
    } else {                  // l = y*nx + x
        base = (l / nx) * pitch + (l % nx);
        stride = ny * pitch;
    }
}

template <int P, int LMAX>
__device__ inline void line_ops(double (&r)[LMAX], int n, int ops, const double* __restrict__ band, double scale,
                                const double* __restrict__ fac) {
    if (ops & OP_GRAM) gram_regs<P, LMAX>(r, n, band, scale);
    if (ops & OP_SOLVE) lu_regs<P, LMAX>(r, n, fac, fac + n * (P - 1), fac + 2 * n * (P - 1));
}

// One mode product over all lines of `axis`, LDS to LDS.
template <int P, int LMAX, int OPS>
__device__ inline void lds_pass(double* buf, int axis, const int d[3], int pitch, const double* __restrict__ band,
                                double scale, const double* __restrict__ fac, int tid, int nthr) {
    const int n = d[2 - axis];
    const int nlines = d[0] * d[1] * d[2] / n;
    auto line = [&](int l) {
        int base, stride;
        line_of(axis, l, d, pitch, base, stride);
        double r[LMAX];
#pragma unroll
        for (int i = 0; i < LMAX; ++i) r[i] = i < n ? buf[base + i * stride] : 0.0;
        line_ops<P, LMAX>(r, n, OPS, band, scale, fac);
#pragma unroll
        for (int i = 0; i < LMAX; ++i)
            if (i < n) buf[base + i * stride] = r[i];
    };
    // one line per thread when the workgroup covers them (the common case: a
    // loop would let the compiler hoist every row's coefficients), else a loop
    if (nlines <= nthr) {
        if (tid < nlines) line(tid);
    } else {
        for (int l = tid; l < nlines; l += nthr) line(l);
    }
}

// First pass of a half step: the curl of the 1-form `src` along each z-line
// of the 2-form component grid od (lanes over x: coalesced global loads),
// with the optional tracking update trk += talpha * curl, written along the
// thread's own line in LDS and read back by the same thread (no barrier), then
// the z-line operations.
template <int P, int LMAX>
__device__ inline void curl_z_pass(double* buf, const double* src, const int64_t soff[3], const int sdims[3][3],
                                   int primal, int c, const int od[3], int pitch, double* trk, double talpha,
                                   int ops, const double* __restrict__ band, double scale,
                                   const double* __restrict__ fac, int tid, int nthr) {
    const int nz = od[0], ny = od[1], nx = od[2];
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    const int zs = ny * pitch;
    for (int l = tid; l < ny * nx; l += nthr) {
        const int y = l / nx, x = l % nx;
        const int base = y * pitch + x;
#pragma unroll 4
        for (int z = 0; z < nz; ++z) {
            double p0, p1, q0, q1;
            diff_pair(src + soff[a2], sdims[a2], primal, a1, z, y, x, p0, p1);
            diff_pair(src + soff[a1], sdims[a1], primal, a2, z, y, x, q0, q1);
            const double u = (p0 - p1) - (q0 - q1);
            if (trk) {
                double* t = trk + (z * ny + y) * nx + x;
                *t = *t + talpha * u;
            }
            buf[base + z * zs] = u;
        }
        double r[LMAX];
#pragma unroll
        for (int z = 0; z < LMAX; ++z) r[z] = z < nz ? buf[base + z * zs] : 0.0;
        line_ops<P, LMAX>(r, nz, ops, band, scale, fac);
#pragma unroll
        for (int z = 0; z < LMAX; ++z)
            if (z < nz) buf[base + z * zs] = r[z];
    }
}

// Last pass of a half step: the line operations along `axis` (1 or 2: lanes
// over x, coalesced) and dst += alpha * result straight from registers.
template <int P, int LMAX>
__device__ inline void final_pass(const double* buf, int axis, const int d[3], int pitch, double* dst, double alpha,
                                  int ops, const double* __restrict__ band, double scale,
                                  const double* __restrict__ fac, int tid, int nthr) {
    const int ny = d[1], nx = d[2];
    const int n = d[2 - axis];
    const int nlines = d[0] * ny * nx / n;
    const int gstride = axis == 1 ? nx : ny * nx;
    for (int l = tid; l < nlines; l += nthr) {
        int base, stride;
        line_of(axis, l, d, pitch, base, stride);
        const int gbase = axis == 1 ? (l / nx) * ny * nx + (l % nx) : l;
        double r[LMAX];
#pragma unroll
        for (int i = 0; i < LMAX; ++i) r[i] = i < n ? buf[base + i * stride] : 0.0;
        line_ops<P, LMAX>(r, n, ops, band, scale, fac);
#pragma unroll
        for (int i0 = 0; i0 < LMAX; i0 += CH) {
            double o[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) o[j] = i0 + j < n ? dst[gbase + (i0 + j) * gstride] : 0.0;
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (i0 + j < n) dst[gbase + (i0 + j) * gstride] = o[j] + alpha * r[i0 + j];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// The y-pass of the e half step: Gram product along y, the tested point
// sources of this line (entries with the line's z and x, subtracted in LDS by
// the thread that owns the line), solve along y.
template <int P, int LMAX>
__device__ inline void y_source_pass(double* buf, const int d[3], int pitch, const double* __restrict__ band,
                                     const double* __restrict__ fac, int c, const SepArgs& A, int b, double th,
                                     int tid, int nthr) {
    const int ny = d[1], nx = d[2];
    const int nlines = d[0] * nx;
    const int k0 = A.n_src > 0 ? A.src_off[b] : 0, k1 = A.n_src > 0 ? A.src_off[b + 1] : 0;
    for (int l = tid; l < nlines; l += nthr) {
        int base, stride;
        line_of(1, l, d, pitch, base, stride);
        const int z = l / nx, x = l % nx;
        double r[LMAX];
#pragma unroll
        for (int i = 0; i < LMAX; ++i) r[i] = i < ny ? buf[base + i * stride] : 0.0;
        gram_regs<P, LMAX>(r, ny, band, 1.0);
#pragma unroll
        for (int i = 0; i < LMAX; ++i)
            if (i < ny) buf[base + i * stride] = r[i];
        bool hit = false;
        for (int k = k0; k < k1; ++k) {
            const double* en = A.src_entries + int64_t(k) * A.entries_per * 5;
            for (int q = 0; q < A.entries_per; ++q) {
                if (int(en[5 * q]) != c || int(en[5 * q + 1]) != z || int(en[5 * q + 3]) != x) continue;
                const double* pr = A.src_prof + 4 * k;
                const double dtt = th - pr[0];
                buf[base + int(en[5 * q + 2]) * stride] -= pr[2] * exp(-dtt * dtt / (2.0 * pr[1] * pr[1])) * en[5 * q + 4];
                hit = true;
            }
        }
        if (hit) {
#pragma unroll
            for (int i = 0; i < LMAX; ++i) r[i] = i < ny ? buf[base + i * stride] : 0.0;
        }
        lu_regs<P, LMAX>(r, ny, fac, fac + ny * (P - 1), fac + 2 * ny * (P - 1));
#pragma unroll
        for (int i = 0; i < LMAX; ++i)
            if (i < ny) buf[base + i * stride] = r[i];
    }
}

__host__ __device__ constexpr int pair_lu(int which_K1, int c, int a) {
    return which_K1 ? (a == c ? F_M : F_G) : (a == c ? F_GT : F_MT);
}

// Two variants of the same half steps (the tuner picks one per space):
// VAR 0, phased: per component a curl phase over all entries into LDS, the
//   mode passes (h: G and K^{-1} along x, y, z; e: G along x, y, z, the
//   sources, K^{-1} along x, y, z), and an update phase over all entries;
// VAR 1, fused passes:
//   h:  z (curl from e, [b -= dt u], G_z, K_z^{-1}) | x (G_x, K_x^{-1}) | y (G_y, K_y^{-1}, h += -dt/mu .)
//   e:  z (curl from h, [d += dt v], G_z / eps) | x (G_x) | y (G_y, - s, K_y^{-1}) | x (K_x^{-1})
//       | z (K_z^{-1}, e += dt .)
// The factors along different axes commute (Kronecker products), so every
// Gram product precedes the source and every solve follows it.
template <int P, int LMAX, int VAR>
__global__ void __launch_bounds__(768) sep_kernel(double* __restrict__ E, double* __restrict__ H,
                                                  const double* __restrict__ gram,
                                                  const double* __restrict__ fac, const SepArgs A) {
    extern __shared__ double buf[];
    const int b = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    double* e = E + int64_t(b) * A.e_stride;
    double* h = H + int64_t(b) * A.h_stride;
    const double t0 = A.t_dev ? *A.t_dev : A.t_start;
    if constexpr (VAR == 0) {
#pragma unroll 1
        for (int step = 0; step < A.nsteps; ++step) {
            // ---- h^{n+1/2} = h^{n-1/2} - dt K~1^{-1} M D^1 e^n   [b -= dt D^1 e] ----
#pragma unroll 1
            for (int c = 0; c < 3; ++c) {
                const int* od = A.hdims[c];
                const int pitch = od[2] | 1;
                curl_to_lds<4>(buf, e, A.e_off, A.edims, 1, c, od, A.track ? h + A.n_h + A.h_off[c] : nullptr, -A.dt,
                               tid, nthr);
                __syncthreads();
#pragma unroll 1
                for (int a = 0; a < 3; ++a) {
                    lds_pass<P, LMAX, OP_GRAM | OP_SOLVE>(buf, a, od, pitch, gram + A.gram_off[space_tag(SP_B, c, a)],
                                                          1.0, fac + A.fac_off[pair_lu(0, c, a)], tid, nthr);
                    __syncthreads();
                }
                update_from_lds<8>(h + A.h_off[c], buf, od, -A.dt * A.inv_mu, tid, nthr);
                __syncthreads();
            }
            // ---- e^{n+1} = e^n + dt K1^{-1} (M~ D~^1 h^{n+1/2} - s(t_{n+1/2}))   [d += dt D~^1 h] ----
            const double th = t0 + (step + 0.5) * A.dt;
#pragma unroll 1
            for (int c = 0; c < 3; ++c) {
                const int* od = A.edims[c];
                const int ny = od[1], pitch = od[2] | 1;
                curl_to_lds<4>(buf, h, A.h_off, A.hdims, 0, c, od, A.track ? e + A.n_e + A.e_off[c] : nullptr, A.dt,
                               tid, nthr);
                __syncthreads();
#pragma unroll 1
                for (int a = 0; a < 3; ++a) {
                    lds_pass<P, LMAX, OP_GRAM>(buf, a, od, pitch, gram + A.gram_off[space_tag(SP_D, c, a)],
                                               a == 2 ? A.inv_eps : 1.0, fac, tid, nthr);
                    __syncthreads();
                }
                // tested point sources, subtracted between the Gram products and the solves
                for (int k = A.n_src > 0 ? A.src_off[b] : 0; k < (A.n_src > 0 ? A.src_off[b + 1] : 0); ++k) {
                    const double* pr = A.src_prof + 4 * k;
                    const double dtt = th - pr[0];
                    const double gt = pr[2] * exp(-dtt * dtt / (2.0 * pr[1] * pr[1]));
                    const double* en = A.src_entries + int64_t(k) * A.entries_per * 5;
                    for (int q = tid; q < A.entries_per; q += nthr)
                        if (int(en[5 * q]) == c)
                            buf[(int(en[5 * q + 1]) * ny + int(en[5 * q + 2])) * pitch + int(en[5 * q + 3])] -=
                                gt * en[5 * q + 4];
                    __syncthreads();
                }
#pragma unroll 1
                for (int a = 2; a >= 0; --a) {
                    lds_pass<P, LMAX, OP_SOLVE>(buf, a, od, pitch, gram, 1.0, fac + A.fac_off[pair_lu(1, c, a)], tid,
                                                nthr);
                    __syncthreads();
                }
                update_from_lds<8>(e + A.e_off[c], buf, od, A.dt, tid, nthr);
                __syncthreads();
            }
        }
    } else {
#pragma unroll 1
        for (int step = 0; step < A.nsteps; ++step) {
            // ---- h^{n+1/2} = h^{n-1/2} - dt K~1^{-1} M D^1 e^n   [b -= dt D^1 e] ----
#pragma unroll 1
            for (int c = 0; c < 3; ++c) {
                const int* od = A.hdims[c];
                const int pitch = od[2] | 1;
                curl_z_pass<P, LMAX>(buf, e, A.e_off, A.edims, 1, c, od, pitch,
                                     A.track ? h + A.n_h + A.h_off[c] : nullptr, -A.dt, OP_GRAM | OP_SOLVE,
                                     gram + A.gram_off[space_tag(SP_B, c, 2)], 1.0, fac + A.fac_off[pair_lu(0, c, 2)],
                                     tid, nthr);
                __syncthreads();
                lds_pass<P, LMAX, OP_GRAM | OP_SOLVE>(buf, 0, od, pitch, gram + A.gram_off[space_tag(SP_B, c, 0)], 1.0,
                                                      fac + A.fac_off[pair_lu(0, c, 0)], tid, nthr);
                __syncthreads();
                final_pass<P, LMAX>(buf, 1, od, pitch, h + A.h_off[c], -A.dt * A.inv_mu, OP_GRAM | OP_SOLVE,
                                    gram + A.gram_off[space_tag(SP_B, c, 1)], 1.0, fac + A.fac_off[pair_lu(0, c, 1)],
                                    tid, nthr);
                __syncthreads();
            }
            // ---- e^{n+1} = e^n + dt K1^{-1} (M~ D~^1 h^{n+1/2} - s(t_{n+1/2}))   [d += dt D~^1 h] ----
            const double th = t0 + (step + 0.5) * A.dt;
#pragma unroll 1
            for (int c = 0; c < 3; ++c) {
                const int* od = A.edims[c];
                const int pitch = od[2] | 1;
                curl_z_pass<P, LMAX>(buf, h, A.h_off, A.hdims, 0, c, od, pitch,
                                     A.track ? e + A.n_e + A.e_off[c] : nullptr, A.dt, OP_GRAM,
                                     gram + A.gram_off[space_tag(SP_D, c, 2)], A.inv_eps, fac, tid, nthr);
                __syncthreads();
                lds_pass<P, LMAX, OP_GRAM>(buf, 0, od, pitch, gram + A.gram_off[space_tag(SP_D, c, 0)], 1.0, fac, tid,
                                           nthr);
                __syncthreads();
                y_source_pass<P, LMAX>(buf, od, pitch, gram + A.gram_off[space_tag(SP_D, c, 1)],
                                       fac + A.fac_off[pair_lu(1, c, 1)], c, A, b, th, tid, nthr);
                __syncthreads();
                lds_pass<P, LMAX, OP_SOLVE>(buf, 0, od, pitch, gram, 1.0, fac + A.fac_off[pair_lu(1, c, 0)], tid, nthr);
                __syncthreads();
                final_pass<P, LMAX>(buf, 2, od, pitch, e + A.e_off[c], A.dt, OP_SOLVE, gram, 1.0,
                                    fac + A.fac_off[pair_lu(1, c, 2)], tid, nthr);
                __syncthreads();
            }
        }
    }
}

}  // namespace

// LDS bytes the separable kernel needs: the largest component tensor of the
// e/d and h/b grids with odd row pitch.
size_t sep_lds_bytes(const int edims[3][3], const int hdims[3][3]) {
    size_t m = 0;
    for (int c = 0; c < 3; ++c) {
        const size_t se = size_t(edims[c][0]) * edims[c][1] * (edims[c][2] | 1);
        const size_t sh = size_t(hdims[c][0]) * hdims[c][1] * (hdims[c][2] | 1);
        m = se > m ? se : m;
        m = sh > m ? sh : m;
    }
    return m * sizeof(double);
}

int sep_line_max(int n_max) { return n_max <= 16 ? 16 : (n_max <= SEP_LINE_MAX ? SEP_LINE_MAX : 0); }

namespace {
template <int PP, int LL, int VV>
hipError_t sep_raise_lds(size_t shm) {
    static size_t done = 0;  // per instantiation: the limit already granted
    if (done >= shm) return hipSuccess;
    const hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(sep_kernel<PP, LL, VV>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
    if (err == hipSuccess) done = shm;
    return err;
}
}  // namespace

#define SEP_DISPATCH(CALL)                                                                       \
    if (p == 2 && lmax == 16) CALL(2, 16)                                                        \
    if (p == 3 && lmax == 16) CALL(3, 16)                                                        \
    if (p == 4 && lmax == 16) CALL(4, 16)                                                        \
    if (p == 2 && lmax == SEP_LINE_MAX) CALL(2, SEP_LINE_MAX)                                    \
    if (p == 3 && lmax == SEP_LINE_MAX) CALL(3, SEP_LINE_MAX)                                    \
    if (p == 4 && lmax == SEP_LINE_MAX) CALL(4, SEP_LINE_MAX)                                    \
    return hipErrorInvalidValue;

hipError_t sep_prepare(int p, int lmax, size_t shm) {
#define PREP(PP, LL)                                                   \
    {                                                                  \
        const hipError_t e0 = sep_raise_lds<PP, LL, 0>(shm);           \
        return e0 != hipSuccess ? e0 : sep_raise_lds<PP, LL, 1>(shm);  \
    }
    SEP_DISPATCH(PREP)
#undef PREP
}

hipError_t launch_sep(int p, int lmax, int variant, double* E, double* H, const double* gram, const double* fac,
                      const SepArgs& a, int batch, int threads, hipStream_t s) {
    const size_t shm = sep_lds_bytes(a.edims, a.hdims);
#define LAUNCH_V(PP, LL, VV)                                                                                   \
    {                                                                                                          \
        const hipError_t err = sep_raise_lds<PP, LL, VV>(shm);                                                 \
        if (err != hipSuccess) return err;                                                                     \
        hipLaunchKernelGGL((sep_kernel<PP, LL, VV>), dim3(batch), dim3(threads), shm, s, E, H, gram, fac, a);  \
        return hipGetLastError();                                                                              \
    }
#define LAUNCH(PP, LL)                      \
    {                                       \
        if (variant == 0) LAUNCH_V(PP, LL, 0) \
        else LAUNCH_V(PP, LL, 1)            \
    }
    SEP_DISPATCH(LAUNCH)
#undef LAUNCH
#undef LAUNCH_V
}

}  // namespace kmx
