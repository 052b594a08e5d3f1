// Host-side set-up of the discrete spaces (runs once per space, not per step):
// knot vectors, Gauss rules, 1D basis tables, the 1D pairing matrices G^ and
// M^ with their banded LU factors, the 2-form metric factor at the Gauss
// points, the projection of initial data and the tested dipole sources.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "kmx_internal.hpp"
#include "setup.hpp"

namespace kmx {

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [-1, 1] by Newton's method on P_n (three-term
// recurrence), started from the Chebyshev-like guess cos(pi (i - 1/4)/(n + 1/2)).
// ---------------------------------------------------------------------------
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged root
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// Knot vectors: Xi (p-open, N uniform elements), Xi' and Xi'' (trimmed).
static std::vector<double> knots_for(int p, int N, int trim) {
    std::vector<double> t;
    for (int i = 0; i < p + 1; ++i) t.push_back(0.0);
    for (int i = 1; i < N; ++i) t.push_back(double(i) / N);
    for (int i = 0; i < p + 1; ++i) t.push_back(1.0);
    return std::vector<double>(t.begin() + trim, t.end() - trim);
}

// Values of the deg+1 B-splines of degree `deg` that are nonzero on knot span
// s (t[s] <= x <= t[s+1]), i.e. B_{s-deg}, ..., B_s, by the triangular
// Cox-de Boor recurrence.
void nonzero_bsplines(const std::vector<double>& t, int s, int deg, double x, double* out) {
    double left[8], right[8];
    out[0] = 1.0;
    for (int j = 1; j <= deg; ++j) {
        left[j] = x - t[s + 1 - j];
        right[j] = t[s + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double tmp = out[r] / (right[r + 1] + left[j - r]);
            out[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        out[j] = saved;
    }
}

// Values of the K(tag) functions of `tag` that are nonzero on element e, at x.
void eval_tag_on_element(const Tables& tb, int tag, int e, double x, double* vals) {
    const int p = tb.p, N = tb.N;
    switch (tag) {
        case PV: {
            auto t = knots_for(p, N, 0);
            nonzero_bsplines(t, p + e, p, x, vals);  // full indices e..e+p
            for (int j = 0; j <= p; ++j) {
                int g = e + j - 1;  // index in the homogeneous space
                if (g < 0 || g >= tb.n0) vals[j] = 0.0;
            }
            break;
        }
        case PF: {
            auto t = knots_for(p, N, 0);
            nonzero_bsplines(t, p + e, p, x, vals);  // full indices e..e+p, none removed
            break;
        }
        case PD:
        case DV: {
            auto t = knots_for(p, N, 1);
            nonzero_bsplines(t, p - 1 + e, p - 1, x, vals);  // indices e..e+p-1
            if (tag == PD)
                for (int j = 0; j < p; ++j) {
                    int g = e + j;
                    vals[j] *= p / (t[g + p] - t[g]);  // Curry-Schoenberg: unit integral
                }
            break;
        }
        case DD: {
            auto t = knots_for(p, N, 2);
            nonzero_bsplines(t, p - 2 + e, p - 2, x, vals);  // indices e..e+p-2
            for (int j = 0; j < p - 1; ++j) {
                int g = e + j;
                vals[j] *= (p - 1) / (t[g + p - 1] - t[g]);
            }
            break;
        }
    }
}

// Banded LU without pivoting of an n x n matrix whose nonzeros lie within
// half bandwidth w.  The 1D pairing matrices are diagonally dominant for
// p <= 3 and, like B-spline Gram matrices, admit elimination without row
// exchanges for the degrees supported here; the solve residual is checked
// against dense solves by the tests.
BandLU band_lu(const std::vector<double>& A, int n, int w) {
    BandLU f;
    f.n = n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (A[i * n + j] != 0.0 && std::abs(i - j) > w)
                throw std::runtime_error("matrix exceeds the expected band");
    f.w = w;
    std::vector<double> a(A);
    f.band.assign(size_t(n) * (2 * w + 1), 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 2 * w + 1; ++k) {
            int j = i - w + k;
            if (j >= 0 && j < n) f.band[i * (2 * w + 1) + k] = A[i * n + j];
        }
    for (int k = 0; k < n; ++k) {
        double piv = a[k * n + k];
        if (piv == 0.0) throw std::runtime_error("zero pivot in banded LU");
        for (int i = k + 1; i <= std::min(n - 1, k + w); ++i) {
            double l = a[i * n + k] / piv;
            a[i * n + k] = l;
            for (int j = k + 1; j <= std::min(n - 1, k + w); ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
    f.L.assign(size_t(n) * w, 0.0);
    f.U.assign(size_t(n) * w, 0.0);
    f.dinv.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        f.dinv[i] = 1.0 / a[i * n + i];
        for (int k = 0; k < w; ++k) {
            if (i - 1 - k >= 0) f.L[i * w + k] = a[i * n + (i - 1 - k)];
            if (i + 1 + k < n) f.U[i * w + k] = a[i * n + (i + 1 + k)];
        }
    }
    return f;
}

void band_solve_host(const BandLU& f, double* x, int64_t stride) {
    const int n = f.n, w = f.w;
    for (int i = 0; i < n; ++i) {
        double s = x[i * stride];
        for (int k = 0; k < w && i - 1 - k >= 0; ++k) s -= f.L[i * w + k] * x[(i - 1 - k) * stride];
        x[i * stride] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i * stride];
        for (int k = 0; k < w && i + 1 + k < n; ++k) s -= f.U[i * w + k] * x[(i + 1 + k) * stride];
        x[i * stride] = s * f.dinv[i];
    }
}

void build_tables(Tables& tb, int p, int N) {
    tb.p = p;
    tb.N = N;
    tb.nq = p + 1;
    tb.n0 = N + p - 2;
    tb.n1 = N + p - 1;
    tb.npad = ((N + TILE - 1) / TILE) * TILE;
    std::vector<double> g, gw;
    gauss_legendre(tb.nq, g, gw);
    const double h = 1.0 / N;
    tb.xq.resize(size_t(N) * tb.nq);
    tb.wq.resize(size_t(N) * tb.nq);
    for (int e = 0; e < N; ++e)
        for (int q = 0; q < tb.nq; ++q) {
            tb.xq[e * tb.nq + q] = (e + 0.5 * (g[q] + 1.0)) * h;
            tb.wq[e * tb.nq + q] = 0.5 * gw[q] * h;
        }
    for (int tag = 0; tag < 4; ++tag) {
        const int K = tag_support(p, tag);
        tb.tab[tag].assign(size_t(tb.npad) * tb.nq * K, 0.0);
        for (int e = 0; e < N; ++e)
            for (int q = 0; q < tb.nq; ++q)
                eval_tag_on_element(tb, tag, e, tb.xq[e * tb.nq + q], &tb.tab[tag][(e * tb.nq + q) * K]);
    }
    tb.tab_pf.assign(size_t(N) * tb.nq * (p + 1), 0.0);
    for (int e = 0; e < N; ++e)
        for (int q = 0; q < tb.nq; ++q)
            eval_tag_on_element(tb, PF, e, tb.xq[e * tb.nq + q], &tb.tab_pf[(e * tb.nq + q) * (p + 1)]);
    // 1D pairing matrices G^ = int Dd^T Pv (n0 x n0), M^ = int Dv^T Pd (n1 x n1)
    const int n0 = tb.n0, n1 = tb.n1;
    tb.G.assign(size_t(n0) * n0, 0.0);
    tb.M.assign(size_t(n1) * n1, 0.0);
    const int Kpv = tag_support(p, PV), Kpd = tag_support(p, PD), Kdd = tag_support(p, DD),
              Kdv = tag_support(p, DV);
    for (int e = 0; e < N; ++e)
        for (int q = 0; q < tb.nq; ++q) {
            const double w = tb.wq[e * tb.nq + q];
            const double* dd = &tb.tab[DD][(e * tb.nq + q) * Kdd];
            const double* pv = &tb.tab[PV][(e * tb.nq + q) * Kpv];
            const double* dv = &tb.tab[DV][(e * tb.nq + q) * Kdv];
            const double* pd = &tb.tab[PD][(e * tb.nq + q) * Kpd];
            for (int i = 0; i < Kdd; ++i)
                for (int j = 0; j < Kpv; ++j) {
                    int r = e + i, c = e + j - 1;
                    if (c >= 0 && c < n0) tb.G[r * n0 + c] += w * dd[i] * pv[j];
                }
            for (int i = 0; i < Kdv; ++i)
                for (int j = 0; j < Kpd; ++j) tb.M[(e + i) * n1 + (e + j)] += w * dv[i] * pd[j];
        }
    std::vector<double> GT(tb.G.size()), MT(tb.M.size());
    for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n0; ++j) GT[j * n0 + i] = tb.G[i * n0 + j];
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) MT[j * n1 + i] = tb.M[i * n1 + j];
    tb.lu[F_G] = band_lu(tb.G, n0, p - 1);
    tb.lu[F_M] = band_lu(tb.M, n1, p - 1);
    tb.lu[F_GT] = band_lu(GT, n0, p - 1);
    tb.lu[F_MT] = band_lu(MT, n1, p - 1);
}

// Jacobian of the map at parametric point xh.
void map_jacobian(const kmx_space* sp, int64_t qp_index, const double xh[3], double J[9]) {
    for (int i = 0; i < 9; ++i) J[i] = (i % 4 == 0) ? 1.0 : 0.0;
    if (sp->map.kind == 1) {
        const double a = sp->map.amplitude;
        const double sx = std::sin(M_PI * xh[0]), sy = std::sin(M_PI * xh[1]), sz = std::sin(M_PI * xh[2]);
        const double cx = std::cos(M_PI * xh[0]), cy = std::cos(M_PI * xh[1]), cz = std::cos(M_PI * xh[2]);
        const double grad[3] = {M_PI * cx * sy * sz, M_PI * sx * cy * sz, M_PI * sx * sy * cz};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J[3 * i + j] += a * grad[j];
    } else if (sp->map.kind == 2) {
        for (int i = 0; i < 9; ++i) J[i] = sp->dF_user[size_t(qp_index) * 9 + i];
    }
}

void map_point(const kmx_space* sp, const double xh[3], double x[3]) {
    for (int i = 0; i < 3; ++i) x[i] = xh[i];
    if (sp->map.kind == 1) {
        const double s = std::sin(M_PI * xh[0]) * std::sin(M_PI * xh[1]) * std::sin(M_PI * xh[2]);
        for (int i = 0; i < 3; ++i) x[i] += sp->map.amplitude * s;
    }
}

static double det3(const double J[9]) {
    return J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
           J[2] * (J[3] * J[7] - J[4] * J[6]);
}

// Element-major quadrature point index.
static inline int64_t qp_index(const Tables& tb, int ez, int ey, int ex, int iz, int iy, int ix) {
    const int64_t N = tb.N, nq = tb.nq;
    return ((((ez * N + ey) * N + ex) * nq + iz) * nq + iy) * nq + ix;
}

// Metric factor w_q DF^T DF / det DF (2-forms) or w_q det DF (DF^T DF)^{-1}
// (1-forms, the covariant pullback) at every Gauss point, laid out per tile of
// TILE^3 elements as [tile][qz][6][qy][qx] with Q = TILE*nq points per tile
// edge; entries 0..5 = (xx, yy, zz, xy, xz, yz).  Padded elements get zeros.
kmx_status build_metric(const kmx_space* sp, std::vector<double>* out, int form) {
    const Tables& tb = sp->tb;
    const int nq = tb.nq, Q = TILE * nq, nt = sp->ntile, N = tb.N;
    if (out) out->assign(size_t(nt) * nt * nt * Q * 6 * Q * Q, 0.0);
    for (int ez = 0; ez < N; ++ez)
        for (int ey = 0; ey < N; ++ey)
            for (int ex = 0; ex < N; ++ex) {
                const int tx = ex / TILE, ty = ey / TILE, tz = ez / TILE;
                const int64_t tile = (int64_t(tz) * nt + ty) * nt + tx;
                for (int iz = 0; iz < nq; ++iz)
                    for (int iy = 0; iy < nq; ++iy)
                        for (int ix = 0; ix < nq; ++ix) {
                            const double xh[3] = {tb.xq[ex * nq + ix], tb.xq[ey * nq + iy], tb.xq[ez * nq + iz]};
                            const double w = tb.wq[ex * nq + ix] * tb.wq[ey * nq + iy] * tb.wq[ez * nq + iz];
                            double J[9];
                            map_jacobian(sp, qp_index(tb, ez, ey, ex, iz, iy, ix), xh, J);
                            const double det = det3(J);
                            if (!(det > 0.0) || !std::isfinite(det)) return KMX_E_GEOMETRY;
                            if (!out) continue;
                            double C[6];
                            const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
                            double S[3][3];
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j) {
                                    double s = 0.0;
                                    for (int r = 0; r < 3; ++r) s += J[3 * r + i] * J[3 * r + j];
                                    S[i][j] = s;
                                }
                            if (form == 2) {
                                for (int k = 0; k < 6; ++k) C[k] = w * S[ii[k]][jj[k]] / det;
                            } else {
                                // det (S^{-1}) = det * adj(S) / det(S), det(S) = det^2
                                for (int k = 0; k < 6; ++k) {
                                    const int i = ii[k], j = jj[k];
                                    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                                    const double cof = S[j1][i1] * S[j2][i2] - S[j1][i2] * S[j2][i1];
                                    C[k] = w * cof / det;
                                }
                            }
                            const int qz = (ez % TILE) * nq + iz, qy = (ey % TILE) * nq + iy,
                                      qx = (ex % TILE) * nq + ix;
                            for (int k = 0; k < 6; ++k)
                                (*out)[((tile * Q + qz) * 6 + k) * Q * Q + qy * Q + qx] = C[k];
                        }
            }
    return KMX_OK;
}

void quad_points(const kmx_space* sp, double* xyz) {
    const Tables& tb = sp->tb;
    const int nq = tb.nq, N = tb.N;
    for (int ez = 0; ez < N; ++ez)
        for (int ey = 0; ey < N; ++ey)
            for (int ex = 0; ex < N; ++ex)
                for (int iz = 0; iz < nq; ++iz)
                    for (int iy = 0; iy < nq; ++iy)
                        for (int ix = 0; ix < nq; ++ix) {
                            const double xh[3] = {tb.xq[ex * nq + ix], tb.xq[ey * nq + iy], tb.xq[ez * nq + iz]};
                            map_point(sp, xh, &xyz[3 * qp_index(tb, ez, ey, ex, iz, iy, ix)]);
                        }
}

// Component dims (nz, ny, nx) and offsets of a form space.
void comp_dims(const kmx_space* sp, int space, int c, int dims[3]) {
    for (int a = 0; a < 3; ++a) {
        int tag = space_tag(space, c, a);
        dims[2 - a] = (tag == PV || tag == DD) ? sp->n0 : sp->n1;
    }
}

int64_t comp_offset(const kmx_space* sp, int space, int c) {
    int64_t o = 0;
    for (int k = 0; k < c; ++k) {
        int d[3];
        comp_dims(sp, space, k, d);
        o += int64_t(d[0]) * d[1] * d[2];
    }
    return o;
}

// form 2: l_i = sum_q w_q eta^_i(q) . (DF^T E0)(q) over the dual 2-form basis;
// form 1: l_i = sum_q w_q eps_e eta^_i(q) . (det DF DF^{-1} E0)(q) over the
// primal 1-form basis (the L^2_eps load vector of the first scheme).
void load_E(const kmx_space* sp, const double* E_qp, std::vector<double>& l, int form) {
    const Tables& tb = sp->tb;
    const int nq = tb.nq, N = tb.N, p = tb.p;
    const int space = form == 1 ? SP_E : SP_D;
    l.assign(sp->n_e, 0.0);
    std::vector<double> F(size_t(nq) * nq * nq * 3);
    for (int ez = 0; ez < N; ++ez)
        for (int ey = 0; ey < N; ++ey)
            for (int ex = 0; ex < N; ++ex) {
                for (int iz = 0; iz < nq; ++iz)
                    for (int iy = 0; iy < nq; ++iy)
                        for (int ix = 0; ix < nq; ++ix) {
                            const int64_t q = qp_index(tb, ez, ey, ex, iz, iy, ix);
                            const double xh[3] = {tb.xq[ex * nq + ix], tb.xq[ey * nq + iy], tb.xq[ez * nq + iz]};
                            const double w = tb.wq[ex * nq + ix] * tb.wq[ey * nq + iy] * tb.wq[ez * nq + iz];
                            double J[9];
                            map_jacobian(sp, q, xh, J);
                            if (form == 1) {
                                // det DF DF^{-1} = adj(DF): row c of the adjugate is the
                                // cross product of the columns c+1 and c+2 of DF
                                const double eps = sp->eps_host.empty()
                                                       ? 1.0
                                                       : sp->eps_host[(size_t(ez) * N + ey) * N + ex];
                                for (int c = 0; c < 3; ++c) {
                                    const int a = (c + 1) % 3, b = (c + 2) % 3;
                                    double s = 0.0;
                                    for (int r = 0; r < 3; ++r) {
                                        const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
                                        const double adj = J[3 * r1 + a] * J[3 * r2 + b] - J[3 * r2 + a] * J[3 * r1 + b];
                                        s += adj * E_qp[3 * q + r];
                                    }
                                    F[((iz * nq + iy) * nq + ix) * 3 + c] = w * eps * s;
                                }
                            } else {
                                for (int c = 0; c < 3; ++c) {
                                    double s = 0.0;
                                    for (int r = 0; r < 3; ++r) s += J[3 * r + c] * E_qp[3 * q + r];
                                    F[((iz * nq + iy) * nq + ix) * 3 + c] = w * s;
                                }
                            }
                        }
                for (int c = 0; c < 3; ++c) {
                    const int tgx = space_tag(space, c, 0), tgy = space_tag(space, c, 1), tgz = space_tag(space, c, 2);
                    const int Kx = tag_support(p, tgx), Ky = tag_support(p, tgy), Kz = tag_support(p, tgz);
                    const int ox = tag_offset(tgx), oy = tag_offset(tgy), oz = tag_offset(tgz);
                    int d[3];
                    comp_dims(sp, space, c, d);
                    const int64_t off = comp_offset(sp, space, c);
                    for (int iz = 0; iz < nq; ++iz)
                        for (int iy = 0; iy < nq; ++iy)
                            for (int ix = 0; ix < nq; ++ix) {
                                const double* bx = &tb.tab[tgx][(ex * nq + ix) * Kx];
                                const double* by = &tb.tab[tgy][(ey * nq + iy) * Ky];
                                const double* bz = &tb.tab[tgz][(ez * nq + iz) * Kz];
                                const double f = F[((iz * nq + iy) * nq + ix) * 3 + c];
                                for (int jz = 0; jz < Kz; ++jz)
                                    for (int jy = 0; jy < Ky; ++jy)
                                        for (int jx = 0; jx < Kx; ++jx) {
                                            // boundary functions of the primal space are not unknowns
                                            const int gz = ez + jz + oz, gy = ey + jy + oy, gx = ex + jx + ox;
                                            if (gz < 0 || gy < 0 || gx < 0 || gz >= d[0] || gy >= d[1] || gx >= d[2])
                                                continue;
                                            l[off + (int64_t(gz) * d[1] + gy) * d[2] + gx] += bz[jz] * by[jy] * bx[jx] * f;
                                        }
                            }
                }
            }
}

// x = K1^{-1} y on the host (per component, per axis banded solves).
void kron_solve_K1_host(const kmx_space* sp, std::vector<double>& y) {
    for (int c = 0; c < 3; ++c) {
        int d[3];
        comp_dims(sp, SP_D, c, d);
        const int nz = d[0], ny = d[1], nx = d[2];
        double* X = y.data() + comp_offset(sp, SP_D, c);
        for (int a = 0; a < 3; ++a) {
            const BandLU& f = sp->tb.lu[a == c ? F_M : F_G];
            if (a == 0)
                for (int z = 0; z < nz; ++z)
                    for (int yy = 0; yy < ny; ++yy) band_solve_host(f, X + (int64_t(z) * ny + yy) * nx, 1);
            else if (a == 1)
                for (int z = 0; z < nz; ++z)
                    for (int x = 0; x < nx; ++x) band_solve_host(f, X + int64_t(z) * ny * nx + x, nx);
            else
                for (int yy = 0; yy < ny; ++yy)
                    for (int x = 0; x < nx; ++x) band_solve_host(f, X + int64_t(yy) * nx + x, int64_t(nx) * ny);
        }
    }
}

// Tested point dipole: entries of s_i = q . DF eta^_i(x0) / (eps det DF) on the
// dual 2-form basis functions whose support contains x0.
void dipole_entries(const kmx_space* sp, const double pos[3], const double q[3],
                    std::vector<DipoleEntry>& out) {
    const Tables& tb = sp->tb;
    const int N = tb.N, p = tb.p;
    int el[3];
    for (int a = 0; a < 3; ++a) el[a] = std::min(std::max(int(std::floor(pos[a] * N)), 0), N - 1);
    double J[9];
    const int64_t qidx = -1;
    if (sp->map.kind == 2) {
        // user Jacobians are only known at quadrature points: use the one of the
        // element's first point
        map_jacobian(sp, qp_index(tb, el[2], el[1], el[0], 0, 0, 0), pos, J);
    } else {
        map_jacobian(sp, qidx, pos, J);
    }
    const double det = det3(J);
    const double inv_eps = sp->inv_eps_host[(int64_t(el[2]) * N + el[1]) * N + el[0]];
    out.clear();
    for (int c = 0; c < 3; ++c) {
        double qc = 0.0;
        for (int r = 0; r < 3; ++r) qc += q[r] * J[3 * r + c];
        const double coef = inv_eps * qc / det;
        double b[3][8];
        int K[3];
        for (int a = 0; a < 3; ++a) {
            const int tag = space_tag(SP_D, c, a);
            K[a] = tag_support(p, tag);
            eval_tag_on_element(tb, tag, el[a], pos[a], b[a]);
        }
        for (int jz = 0; jz < K[2]; ++jz)
            for (int jy = 0; jy < K[1]; ++jy)
                for (int jx = 0; jx < K[0]; ++jx)
                    out.push_back({c, el[2] + jz, el[1] + jy, el[0] + jx, coef * b[2][jz] * b[1][jy] * b[0][jx]});
    }
}

}  // namespace kmx
