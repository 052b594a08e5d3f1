// Host paths of the library built with the address and undefined-behaviour
// sanitizers (no GPU is touched): 1D tables and factors, the metric and load
// vectors, the host Kronecker solve, tested dipoles, the trace fit and the
// lifting vectors, on small spaces of every degree.  Exits non-zero (the
// sanitizers abort) on an invalid access or undefined behaviour, or when a
// result is not finite or a consistency check fails.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2302_04979_amd/csrc/kernels.hpp"
#include "../../paper_2302_04979_amd/csrc/setup.hpp"

using namespace kmx;

static int fails = 0;
static void check(bool ok, const char* what, int p, int N) {
    if (!ok) {
        std::fprintf(stderr, "check failed: %s (p=%d N=%d)\n", what, p, N);
        ++fails;
    }
}

static void host_space(kmx_space& sp, int p, int N, int kind) {
    sp.p = p;
    sp.N = N;
    sp.nq = p + 1;
    sp.n0 = N + p - 2;
    sp.n1 = N + p - 1;
    sp.ntile = (N + TILE - 1) / TILE;
    sp.npad = sp.ntile * TILE;
    sp.n_e = int64_t(3) * sp.n1 * sp.n0 * sp.n0;
    sp.n_h = int64_t(3) * sp.n0 * sp.n1 * sp.n1;
    sp.n_qp = int64_t(N) * N * N * sp.nq * sp.nq * sp.nq;
    sp.map.kind = kind;
    sp.map.amplitude = kind == 1 ? 0.08 : 0.0;
    build_tables(sp.tb, p, N);
    sp.inv_eps_host.assign(size_t(N) * N * N, 0.5);
    sp.inv_mu_host.assign(size_t(N) * N * N, 1.0);
}

int main() {
    for (int p = 2; p <= 4; ++p)
        for (int N : {1, 3, 5}) {
            kmx_space sp;
            host_space(sp, p, N, 1);
            std::vector<double> metric;
            check(build_metric(&sp, &metric, 2) == KMX_OK, "metric (2-forms)", p, N);
            check(build_metric(&sp, &metric, 1) == KMX_OK, "metric (1-forms)", p, N);
            // load vector of a constant field, then the host solve
            std::vector<double> E(size_t(3) * sp.n_qp, 0.0), l;
            for (int64_t q = 0; q < sp.n_qp; ++q) E[3 * q + 2] = 1.0;
            load_E(&sp, E.data(), l, 2);
            kron_solve_K1_host(&sp, l);
            bool finite = true;
            for (double v : l) finite = finite && std::isfinite(v);
            check(finite && int64_t(l.size()) == sp.n_e, "projection", p, N);
            std::vector<double> l1;
            load_E(&sp, E.data(), l1, 1);
            check(int64_t(l1.size()) == sp.n_e, "1-form load", p, N);
            // a dipole at an interior point and at a corner
            std::vector<DipoleEntry> ent;
            const double pos[3] = {0.37, 0.61, 0.23}, q[3] = {0.3, -0.5, 0.8};
            dipole_entries(&sp, pos, q, ent);
            check(!ent.empty(), "dipole", p, N);
            const double corner[3] = {1.0, 0.0, 1.0};
            dipole_entries(&sp, corner, q, ent);
            // the trace fit returns the boundary coefficients of a whole-space
            // field from its own trace, and the lifting vectors are finite
            const int64_t nf = full_size(&sp, 1);
            std::vector<double> ef(nf);
            for (int64_t i = 0; i < nf; ++i) ef[i] = std::sin(0.7 * double(i) + 0.3);
            const int Q = N * sp.nq;
            std::vector<double> faces(size_t(6) * Q * Q * 3, 0.0);
            for (int a = 0; a < 3; ++a)
                for (int s = 0; s < 2; ++s) {
                    const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
                    for (int iv = 0; iv < Q; ++iv)
                        for (int iu = 0; iu < Q; ++iu) {
                            double xh[3];
                            xh[a] = double(s);
                            xh[u] = sp.tb.xq[iu];
                            xh[v] = sp.tb.xq[iv];
                            for (int c = 0; c < 3; ++c) {
                                int d[3];
                                full_dims(&sp, 1, c, d);
                                const double* F = ef.data() + full_offset(&sp, 1, c);
                                double val = 0.0;
                                // sum of the whole-space basis: element of each coordinate
                                int el[3];
                                double b[3][6];
                                int K[3];
                                for (int k = 0; k < 3; ++k) {
                                    el[k] = std::min(int(xh[k] * N), N - 1);
                                    const int tag = k == c ? PD : PF;
                                    K[k] = tag_support(p, tag);
                                    eval_tag_on_element(sp.tb, tag, el[k], xh[k], b[k]);
                                }
                                for (int jz = 0; jz < K[2]; ++jz)
                                    for (int jy = 0; jy < K[1]; ++jy)
                                        for (int jx = 0; jx < K[0]; ++jx)
                                            val += b[2][jz] * b[1][jy] * b[0][jx] *
                                                   F[(int64_t(el[2] + jz) * d[1] + el[1] + jy) * d[2] + el[0] + jx];
                                faces[((size_t(2 * a + s) * Q + iv) * Q + iu) * 3 + c] = val;
                            }
                        }
                }
            std::vector<double> eb(nf, 0.0);
            const int it = boundary_fit(&sp, faces.data(), eb.data(), 1e-14, 5000);
            check(it >= 0, "trace fit converged", p, N);
            double err = 0.0, mag = 0.0;
            for (int c = 0; c < 3; ++c) {
                int d[3];
                full_dims(&sp, 1, c, d);
                const int64_t o = full_offset(&sp, 1, c);
                for (int z = 0; z < d[0]; ++z)
                    for (int y = 0; y < d[1]; ++y)
                        for (int x = 0; x < d[2]; ++x) {
                            const int idx[3] = {x, y, z};
                            bool bnd = false;
                            for (int k = 0; k < 3; ++k)
                                if (k != c && (idx[k] == 0 || idx[k] == sp.n0 + 1)) bnd = true;
                            const int64_t i = o + (int64_t(z) * d[1] + y) * d[2] + x;
                            if (bnd) {
                                err = std::fmax(err, std::fabs(eb[i] - ef[i]));
                                mag = std::fmax(mag, std::fabs(ef[i]));
                            }
                        }
            }
            check(err <= 1e-10 * mag, "trace fit exact on a discrete trace", p, N);
            std::vector<double> vh, ve;
            lifting_vectors(&sp, eb.data(), vh, ve);
            finite = int64_t(vh.size()) == sp.n_h && int64_t(ve.size()) == sp.n_e;
            for (double x : vh) finite = finite && std::isfinite(x);
            for (double x : ve) finite = finite && std::isfinite(x);
            check(finite, "lifting vectors", p, N);
        }
    std::printf("host checks: %d failures\n", fails);
    return fails == 0 ? 0 : 1;
}
