// Host set-up routines (setup.hip).
#pragma once

#include <vector>

#include "kmx_internal.hpp"

namespace kmx {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// the deg + 1 B-splines of degree deg on knots t nonzero on span s, at x
void nonzero_bsplines(const std::vector<double>& t, int s, int deg, double x, double* out);
void eval_tag_on_element(const Tables& tb, int tag, int e, double x, double* vals);
BandLU band_lu(const std::vector<double>& A, int n, int w);
void band_solve_host(const BandLU& f, double* x, int64_t stride);
void build_tables(Tables& tb, int p, int N);
void map_jacobian(const kmx_space* sp, int64_t qp_index, const double xh[3], double J[9]);
void map_point(const kmx_space* sp, const double xh[3], double x[3]);
// form 2: w DF^T DF / det DF; form 1: w det DF (DF^T DF)^{-1}.  out = nullptr: check det DF only
kmx_status build_metric(const kmx_space* sp, std::vector<double>* out, int form = 2);
void quad_points(const kmx_space* sp, double* xyz);
void comp_dims(const kmx_space* sp, int space, int c, int dims[3]);
int64_t comp_offset(const kmx_space* sp, int space, int c);
void load_E(const kmx_space* sp, const double* E_qp, std::vector<double>& l, int form = 2);
void kron_solve_K1_host(const kmx_space* sp, std::vector<double>& y);
void dipole_entries(const kmx_space* sp, const double pos[3], const double q[3],
                    std::vector<DipoleEntry>& out);

}  // namespace kmx
