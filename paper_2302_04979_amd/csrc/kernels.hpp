// Kernel launch interfaces (kernels.hip).
#pragma once

#include "kmx_internal.hpp"

namespace kmx {

// Mass apply y = M x (or M D x with the curl fused), written as per-tile
// partial sums ("patches") that the solve kernels gather.
struct MassArgs {
    const double* src;          // input field of batch member 0
    int64_t src_stride;         // distance between batch members
    double* patch;              // patch buffer of batch member 0
    int64_t patch_stride;
    const double* metric;       // w_q DF^T DF / det DF, tile layout (metric_mode 0)
    int metric_mode;            // 0 stored metric, 1 recomputed for the sine map
    int waves4;                 // 1: the variant compiled for four waves per SIMD (p <= 3)
    hipEvent_t prof_start;      // profiling: stamped when the kernel starts / ends, or nullptr
    hipEvent_t prof_stop;
    double amp;                 // map amplitude a (metric_mode 1)
    const double* axis_tab;     // [sin | cos | weight] at the npad*nq Gauss points of an axis
    const double* inv_gamma;    // [npad^3] per-element 1/eps or 1/mu, or nullptr
    const double* tab;          // concatenated 1D tables
    int64_t tab_off[4];
    int ntile, npad, n0, n1;
    int64_t src_comp_off[3];
    int src_dims[3][3];         // [c][z, y, x] of the source space
    int64_t patch_comp_off[3];  // per component, within one field's patches
    // optional fused tracking update of the 2-form: track += track_alpha * (curl
    // of the input), each entry written by the one tile that owns it
    double* track;
    int64_t track_stride;
    double track_alpha;
    int64_t track_comp_off[3];
    int track_dims[3][3];
};

// Sum the overlapping tile patches of a mass apply into a field.
struct GatherArgs {
    const double* patch;
    int64_t patch_stride;
    int64_t patch_comp_off[3];
    double* out;
    int64_t out_stride;
    int64_t comp_off[3];
    int dims[3][3];
    int ntile;
    // optional: acc += acc_alpha * (the gathered field), same layout
    double* acc;
    int64_t acc_stride;
    double acc_alpha;
};

// Read a field, subtract point sources, solve (or apply) along x and y.
struct XYArgs {
    const double* in;
    int64_t in_stride;
    double* out;
    int64_t out_stride;
    int64_t comp_off[3];        // component offsets (same for in and out)
    int dims[3][3];             // [c][z, y, x]
    const double* fac;          // banded factor sets
    int64_t fac_off[8];
    int fac_id[3][3];           // [c][axis] factor id; axis 2 unused here
    // point sources (tested dipoles); n_src = 0 when none
    const double* src_entries;  // [n_src][entries_per][5] = comp, iz, iy, ix, value
    const double* src_prof;     // [n_src][4] = t0, sigma, amp, batch
    const int* src_off;         // [batch+1] dipoles of each batch member (sorted)
    int n_src, entries_per;
    double t_src;               // source time = (t_dev ? *t_dev : 0) + t_src
    const double* t_dev;
    int solve;                  // line operation: 0 none (copy), 1 solve, 2 banded apply
};

// Solve along z and finish: out = (accumulate ? out : 0) + alpha * x.
struct ZArgs {
    const double* in;
    int64_t in_stride;
    double* out;
    int64_t out_stride;
    int64_t comp_off[3];
    int dims[3][3];
    const double* fac;
    int64_t fac_off[8];
    int fac_id[3];
    double alpha;
    int accumulate;
    int solve;                  // line operation along z: 0 none, 1 solve, 2 banded apply
};

struct CurlArgs {
    const double* in;
    int64_t in_stride;
    double* out;
    int64_t out_stride;
    int64_t in_comp_off[3], out_comp_off[3];
    int in_dims[3][3], out_dims[3][3];
    double alpha, beta;         // out = beta * out + alpha * curl(in)
    int primal;
};

// All three energy terms in one launch (K v formed plane-block by plane-block).
struct EnergyFusedArgs {
    const double* E;            // [e | d] per batch member
    const double* H;            // [h | b]
    int64_t n_e, n_h;
    int64_t e_comp_off[3], h_comp_off[3];
    int e_dims[3][3], h_dims[3][3];
    const double* fac;          // banded factor sets (their stored matrices are used)
    int64_t fac_off[8];
    int fac_id[2][3][3];        // [term group][c][axis]: K1 factors, K~1 factors
    int nb[2];                  // blocks of the first term and of the other two
    int cb[2][3];               // blocks per component
    double* partial;            // [batch][nb0 + nb1][3]
};

// Energy terms of tracked states from the images w_e = K1 e and w_h = K~1 h
// that the step keeps: per block d . w_e, b . w_h and w_h . D^1 e.
struct EnergyDotsArgs {
    const double* E;            // [e | d] per batch member
    const double* H;            // [h | b]
    const double* we;           // K1 e per member (stride n_e)
    const double* wh;           // K~1 h per member (stride n_h)
    int64_t n_e, n_h;
    int64_t e_comp_off[3], h_comp_off[3];
    int e_dims[3][3], h_dims[3][3];
    double* partial;            // [batch][ENERGY_DOT_WORKERS][3]
    // optional: the previous step's partials, finished into prev_out[batch]
    // by one extra workgroup of the same launch (NULL: none)
    const double* prev_partial;
    double* prev_out;
    double prev_dt;
};

struct PairGradArgs {           // per-element metric pairing of lam and D~^1 h
    const double* lam;
    int64_t lam_comp_off[3];
    int lam_dims[3][3];
    const double* h;
    int64_t h_comp_off[3];
    int h_dims[3][3];
    const double* metric;
    int metric_mode;
    double amp;
    const double* axis_tab;
    const double* inv_eps;      // [npad^3]
    const double* tab;
    int64_t tab_off[4];
    int ntile, npad, n0, n1, N;
    double coef;
    double* grad;               // [N^3], x fastest
};

// Persistent leapfrog of separable spaces (identity map, uniform eps and mu):
// one workgroup per batch member runs all nsteps with the component tensors
// in LDS.  Fields are passed as kernel arguments of their own.
constexpr int SEP_LINE_MAX = 28;   // longest line (n0, n1) the kernel holds in registers
constexpr int SEP_MAX_THREADS = 768;  // launch bound of the separable kernel
struct SepArgs {
    int64_t e_stride, h_stride;    // distance between batch members (doubled with tracking)
    int64_t n_e, n_h;              // offset of d inside E and of b inside H
    int track;
    int64_t e_off[3], h_off[3];    // component offsets of the e/d and h/b spaces
    int edims[3][3], hdims[3][3];  // [c][z, y, x]
    int64_t gram_off[4];           // per tag: n rows of 2p+1 band entries (half width p)
    int64_t fac_off[4];            // banded LU of G^, M^, G^T, M^T: [L | U | dinv | band]
    double inv_mu, inv_eps, dt;
    int nsteps;
    double t_start;                // source time of step n: (t_dev ? *t_dev : t_start) + (n + 1/2) dt
    const double* t_dev;
    const double* src_entries;     // as XYArgs
    const double* src_prof;
    const int* src_off;
    int n_src, entries_per;
};
size_t sep_lds_bytes(const int edims[3][3], const int hdims[3][3]);
int sep_line_max(int n_max);       // register line length for lines up to n_max, 0 if too long
hipError_t sep_prepare(int p, int lmax, size_t shm);   // grant the kernel its LDS (outside graph capture)
hipError_t launch_sep(int p, int lmax, int variant, double* E, double* H, const double* gram, const double* fac,
                      const SepArgs& a, int batch, int threads, hipStream_t s);

// Mode-n product of every component of a field with a dense FP32 factor on
// the matrix cores (mixed-precision solves).
struct ModeArgs {
    const void* in;             // FP64 (in_f64) or FP32 field, batch member 0
    int in_f64;
    int64_t in_stride;
    void* out;
    int out_kind;               // 0 FP32 store, 1 FP64 store, 2 FP64 out += alpha * result
    int64_t out_stride;
    double alpha;
    int64_t comp_off[3];        // same layout for in and out
    int dims[3][3];             // [c][z, y, x]
    const float* A;             // dense n x n FP32 factors, row-major
    int64_t A_off[3];           // factor of each component along `axis`
    int axis;
};
int mode_line_max();
void launch_mode(const ModeArgs& a, int batch, hipStream_t s);

// Dense FP64 solves with the inverse 1D factors on the matrix cores: the plane
// pass Y = B_y X B_x^T (less the point sources) and the z pass
// out = (accumulate ? out : 0) + alpha B_z X.
constexpr int DENSE_NMAX = 80;  // longest line
struct DenseArgs {
    const double* in;
    int64_t in_stride;
    double* out;
    int64_t out_stride;
    int64_t comp_off[3];        // same layout for in and out
    int dims[3][3];             // [c][z, y, x]
    const double* frag;         // inverse factors in MFMA operand order
    int64_t frag_off[3][3];     // [c][axis]
    double alpha;               // z pass
    int accumulate;
    const double* src_entries;  // point sources, plane pass (as XYArgs)
    const double* src_prof;
    const int* src_off;
    int n_src, entries_per;
    double t_src;
    const double* t_dev;
};
int64_t dense_frag_doubles(int n);                           // size of one operand-order factor
void dense_fragments(const double* B, int n, double* frag);  // row-major n x n -> operand order
size_t dense_lds_bytes(const int dims[3][3]);                // LDS of the larger of the two kernels
hipError_t dense_prepare(size_t shm);                        // grant the kernels their LDS (outside capture)
void launch_dense_xy(const DenseArgs& a, int batch, hipStream_t s);
void launch_dense_z(const DenseArgs& a, int batch, hipStream_t s);
void launch_strided_axpy(const double* x, int64_t xs, double* y, int64_t ys, int64_t n, double alpha, int batch,
                         hipStream_t s);

void launch_mass(int p, int space, bool curl, const MassArgs& a, int batch, hipStream_t s);
void launch_curlT(const CurlArgs& a, int64_t n_out, int batch, hipStream_t s);
void launch_csr(const int* rowptr, const int* col, const double* val, const double* x, double* out,
                const int* out_index, int nrows, double alpha, double beta, hipStream_t s);
void launch_residual(const double* obs, const double* data, double* r, int64_t n, double* partial, int nblocks,
                     hipStream_t s);
void launch_source_grad(const double* entries, const double* prof, const int* elem, int n_src, int entries_per,
                        const double* lam, const int64_t* comp_off_dev, const int* dims_dev,
                        const double* src_inv_eps, double t, double coef, double* grad, hipStream_t s);
void launch_pair_grad(int p, const PairGradArgs& a, hipStream_t s);
void launch_gather(int p, int space, const GatherArgs& a, int64_t n, int batch, hipStream_t s);
void launch_xy(int p, const XYArgs& a, int batch, hipStream_t s);
void launch_z(int p, const ZArgs& a, int batch, hipStream_t s);
void launch_curl(const CurlArgs& a, int64_t n_out, int batch, hipStream_t s);
void launch_energy_fused(int p, const EnergyFusedArgs& a, int batch, hipStream_t s);
// y -= g(t) P for every batch member (stride y_stride; pattern stride p_stride,
// 0 when all members share one), g the sampled series at t = (*t_dev or 0) + t_src
void launch_pattern_source(double* y, int64_t y_stride, const double* P, int64_t p_stride, int64_t n,
                           const double* series, int m, double t0, double h, const double* t_dev, double t_src,
                           int batch, hipStream_t s);
constexpr int ENERGY_DOT_BLOCKS = 2048;  // blocks per member of the dot kernel
constexpr int ENERGY_DOT_WORKERS = ENERGY_DOT_BLOCKS - 1;  // the first block finishes the previous step
constexpr int ENERGY_DOT_UNROLL = 1;     // entries per thread and loop round
constexpr int ENERGY_DOT_EBLOCKS = 768;  // of the working blocks, those that take the d . w_e items
void launch_energy_dots(const EnergyDotsArgs& a, int batch, hipStream_t s);
int energy_fused_blocks(const int dims[3][3], int cb[3]);
// out[b*out_stride] (+ step offset) from the energy partials
void launch_energy_final(const double* partial, int nblocks, double dt, int batch, double* out,
                         int64_t out_stride, hipStream_t s);
// partial dot products x.y per batch member -> partial[b][nblocks]
void launch_dot(const double* x, const double* y, int64_t n, int64_t stride, int batch,
                double* partial, int nblocks, hipStream_t s);
void launch_sum_final(const double* partial, int nblocks, int batch, double* out, hipStream_t s);
// y = a*x + b*y with device scalars a = sa[0]*ka, b = kb (sa may be null => 1)
void launch_axpby(const double* x, double* y, int64_t n, double ka, const double* sa, double kb,
                  hipStream_t s);
// partial[2 * nblocks] scratch; out0 = r.r, out1 = r.z (device scalars)
void launch_dot2(const double* r, const double* z, int64_t n, double* partial, int nblocks, double* out0,
                 double* out1, hipStream_t s);
// phase 0: x += (num/den) p, r -= (num/den) Ap; phase 1: p = z + (num/den) p
void launch_cg2(double* x, double* r, double* pdir, const double* Ap, const double* z, int64_t n, const double* num,
                const double* den, int phase, hipStream_t s);
void launch_cg_update(double* x, double* r, double* pdir, const double* Ap, const double* z,
                      int64_t n, const double* scal, int phase, hipStream_t s);

void launch_advance_time(double* t, double dt, hipStream_t s);
// Lifting terms of non-homogeneous tangential data: g_j(t) = amp_j cos(omega_j t + phase_j)
constexpr int KMX_LIFT_MAX = 8;
struct LiftTerms {
    int n;
    double amp[KMX_LIFT_MAX], omega[KMX_LIFT_MAX], phase[KMX_LIFT_MAX];
};
// whole primal spaces X^1_h (form 1) and X^2_h (form 2): component dims,
// offsets and sizes
void full_dims(const kmx_space* sp, int form, int c, int d[3]);
int64_t full_offset(const kmx_space* sp, int form, int c);
int64_t full_size(const kmx_space* sp, int form);
// v_h = K~1^{-1} M_{0,f} D^1_f e_b and v_e = K1^{-1} (K1)_b e_b (host, FP64)
void lifting_vectors(const kmx_space* sp, const double* eb_full, std::vector<double>& vh, std::vector<double>& ve);
// least-squares trace fit of the boundary coefficients; returns the CG
// iterations, or -1 when tol was not reached within max_iter
int boundary_fit(const kmx_space* sp, const double* Eh_faces, double* eb_full, double tol, int max_iter);
// out += the lifting's contribution to one half step (mode 0: h, 1: e)
void launch_lift(double* out, int64_t out_stride, const double* v, int64_t n, const LiftTerms& T, double t_base,
                 double t_step, const double* t_dev, double dt, int mode, int batch, hipStream_t s);
// x[0..n) = v (a kernel, so that graph captures hold no memset node)
void launch_fill(double* x, int64_t n, double v, hipStream_t s);

int mass_threads(int p);
int64_t patch_size(int p, int space, int ntile, int64_t comp_off[3]);

}  // namespace kmx
