// Internal definitions shared by the host set-up code and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/kronmaxwell.h"

namespace kmx {

// Elements per tile edge of the mass-apply kernel; tiles are TILE^3 elements.
constexpr int TILE = 4;

// 1D basis tags (Section 2.3 / 4.1):
//   PV primal value S_p(Xi) minus its two boundary functions (dim n0)
//   PD primal derivative, Curry-Schoenberg basis of S_{p-1}(Xi') (dim n1)
//   DV dual value, B-splines of S_{p-1}(Xi') (dim n1)
//   DD dual derivative, Curry-Schoenberg basis of S_{p-2}(Xi'') (dim n0)
enum Tag { PV = 0, PD = 1, DV = 2, DD = 3 };
// The whole S_p(Xi) basis (Pv with its two boundary functions kept), only for
// non-homogeneous boundary data; N + p functions, e .. e + p nonzero on element e.
constexpr int PF = 4;

// Number of basis functions of a tag that are nonzero on one element.
__host__ __device__ constexpr int tag_support(int p, int tag) {
    return (tag == PV || tag == PF) ? p + 1 : (tag == DD ? p - 1 : p);
}
// Global index of local function j on element e is e + j + tag_offset.
__host__ __device__ constexpr int tag_offset(int tag) { return tag == PV ? -1 : 0; }

// Form spaces: component c, axis a -> tag.
enum Space { SP_E = 0, SP_B = 1, SP_H = 2, SP_D = 3 };
__host__ __device__ constexpr int space_tag(int space, int c, int a) {
    return space == SP_E ? (a == c ? PD : PV)
         : space == SP_B ? (a == c ? PV : PD)
         : space == SP_H ? (a == c ? DD : DV)
                         : (a == c ? DV : DD);
}

// Banded LU factors (no pivoting) of an n x n matrix with half bandwidth w,
// stored per row: L[i*w + k] = l(i, i-1-k), U[i*w + k] = u(i, i+1+k),
// dinv[i] = 1/u(i,i); band[i*(2w+1) + k] = a(i, i-w+k) (the matrix itself).
struct BandLU {
    int n = 0, w = 0;
    std::vector<double> L, U, dinv, band;
};

// Device copy of one set of banded factors: contiguous [L | U | dinv | band].
struct DevBand {
    const double* L;
    const double* U;
    const double* dinv;
    const double* band;
    int n, w;
};

// 1D factor ids: G^, M^, G^T, M^T.
enum Fac { F_G = 0, F_M = 1, F_GT = 2, F_MT = 3 };

struct DipoleEntry {   // one nonzero of a tested dipole source
    int comp, iz, iy, ix;
    double val;
};

struct Tables {        // host-side 1D data
    int p = 0, N = 0, nq = 0, n0 = 0, n1 = 0, npad = 0;
    std::vector<double> xq, wq;                 // global Gauss points / weights (N*nq)
    std::vector<double> tab[4];                 // [npad][nq][K(tag)] values at Gauss points
    std::vector<double> tab_pf;                 // [N][nq][p+1] the whole S_p basis (Pv with its
                                                // boundary functions), for boundary data
    std::vector<double> G, M;                   // dense n0 x n0 and n1 x n1
    BandLU lu[4];                               // factors of G, M, G^T, M^T
};

}  // namespace kmx

struct kmx_source {
    kmx_space* sp = nullptr;
    int n = 0;
    int batch_max = 0;                 // 1 + largest batch index
    double* d_entries = nullptr;       // device: per dipole, ENTRIES x {comp,iz,iy,ix,val} as doubles
    double* d_prof = nullptr;          // device: per dipole {t0, sigma, amp, batch}, then batch offsets
    int entries_per = 0;
    int* d_elem = nullptr;             // device: element (x fastest, N^3) holding each dipole
    double* d_inv_eps = nullptr;       // device: 1/eps of that element at creation
    int64_t* d_comp_off = nullptr;     // device: component offsets of the dual 2-form space
    int* d_dims = nullptr;             // device: [3][3] dims of the dual 2-form space
    // kind 1: a dense pattern s (npat patterns of n_e entries: one for every
    // member, or one per member) times a sampled time series g
    int kind = 0;
    int npat = 0, nsamples = 0;
    double ts0 = 0.0, tsh = 0.0;       // sample k at ts0 + k tsh
    double* d_pattern = nullptr;
    double* d_series = nullptr;
};

struct kmx_graph {
    kmx_space* sp = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int nsteps = 0;
};

struct kmx_probes {
    kmx_space* sp = nullptr;
    int n = 0;                         // probes; rows of P = 3 n
    int *d_rowptr = nullptr, *d_col = nullptr;
    double* d_val = nullptr;           // P (rows: probe, physical component; columns: e dofs)
    int ntrows = 0;
    int *d_trowptr = nullptr, *d_tcol = nullptr, *d_tidx = nullptr;
    double* d_tval = nullptr;          // P^T restricted to the e dofs it touches
};

struct kmx_space {
    int p = 0, N = 0, nq = 0, n0 = 0, n1 = 0;
    int npad = 0, ntile = 0;           // padded element count and tiles per axis
    int max_batch = 1;
    int precision = 0;
    int device = 0;                    // HIP device the space was created on
    int64_t n_e = 0, n_h = 0, n_qp = 0;
    kmx::Tables tb;
    kmx_map map{};
    std::vector<double> inv_eps_host, inv_mu_host;   // [N^3] x fastest
    std::vector<double> dF_user;                      // kind 2 copy
    // device data
    double* d_tab = nullptr;           // 4 tag tables concatenated
    int64_t tab_off[4] = {0, 0, 0, 0};
    double* d_metric = nullptr;        // w_q DF^T DF / det DF, tile layout (metric_mode 0)
    int metric_mode = 0;               // 0 stored metric, 1 recomputed in the mass kernel
    double* d_axis_tab = nullptr;      // sin, cos, weight at the Gauss points of an axis
    double* d_inv_eps = nullptr;       // [npad^3]
    double* d_inv_mu = nullptr;        // [npad^3]
    double* d_fac = nullptr;           // 4 banded factor sets
    int64_t fac_off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double* d_patch = nullptr;         // mass-apply partial outputs
    int64_t patch_per_field = 0;
    double* d_tmp = nullptr;           // field-sized scratch [max_batch][max(n_e,n_h)]
    double* d_tmp2 = nullptr;          // second field-sized scratch
    double* d_we = nullptr;            // per-step energy: K1 e per member [max_batch][n_e]
    double* d_wh = nullptr;            // per-step energy: K~1 h per member [max_batch][n_h]
    double* d_red = nullptr;           // reduction partials
    int64_t red_len = 0;
    double* d_scal = nullptr;          // small device scalars
    double* d_time = nullptr;          // device time read by graph-captured steps
    // separable plan (identity map, uniform materials): 1D Gram bands per tag
    double* d_gram = nullptr;          // per tag: n rows x (2p+1), half width p
    int64_t gram_off[4] = {0, 0, 0, 0};
    bool uniform_eps = true, uniform_mu = true;
    double eps_value = 1.0, mu_value = 1.0;   // 1/eps and 1/mu when uniform
    int max_lds = 0;                   // device limit of LDS bytes per workgroup
    int plan_kind = -1;                // -1 automatic, KMX_PLAN_TILED, KMX_PLAN_SEPARABLE
    int plan_threads = 768;            // workgroup size of the separable kernel
    int mass_waves4 = 0;               // tiled plans: mass kernel variant for four waves per SIMD
    // mixed-precision solves (precision & KMX_MIXED): dense FP32 inverses of
    // the four 1D pairing factors and working fields
    float* d_inv32 = nullptr;          // [G^-1 | M^-1 | G^-T | M^-T], row-major
    int64_t inv32_off[4] = {0, 0, 0, 0};
    double *d_mx = nullptr, *d_mr = nullptr, *d_my = nullptr;   // FP64 [max_batch][nfield]
    float *d_m32a = nullptr, *d_m32b = nullptr;                  // FP32 [max_batch][nfield]
    int refine_steps = 2;              // refinement corrections after the first FP32 solve
    // dense FP64 inverses of the four 1D pairing factors (tiled-dense plan)
    double* d_frag64 = nullptr;        // FP64 inverse factors in MFMA operand order (tiled-dense plan)
    // [0..3] inverses of G^, M^, G^T, M^T; [4..7] G^, M^, G^T, M^T themselves
    // (first-scheme pairing applies)
    int64_t frag64_off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int dense_ok = 0;                  // the dense kernels' LDS fits the device
    // first scheme (1-form mass solves), set up at its first use
    std::vector<double> eps_host, mu_host;   // [N^3] eps and mu as given (empty: 1)
    double* d_eps = nullptr;           // [npad^3] eps (the 1-form masses multiply)
    double* d_mu = nullptr;            // [npad^3] mu
    double* d_metric1 = nullptr;       // w_q det DF (DF^T DF)^{-1}, tile layout (metric_mode 0)
    double* d_s1 = nullptr;            // scheme-1 work vectors, S1_VECS x max(n_e, n_h)
    double* d_frag_pre = nullptr;      // scheme-1 preconditioner: inverse weighted 1D Grams, operand order
    int64_t frag_pre_off[2][3][3] = {};  // [E, H][component][axis]
    int s1_ready = 0;                  // d_eps / d_mu hold the current materials
    double* h_rr = nullptr;            // pinned host copies of the CG residual norms (ring of 2)
    hipEvent_t s1_ev[2] = {nullptr, nullptr};  // marks the copies
    hipStream_t capture_stream = nullptr;
    int live_graphs = 0;               // graphs captured on this space and not yet destroyed
    // lifting of non-homogeneous tangential E data (kmx_set_lifting)
    int lift_n = 0;
    double *d_lift_vh = nullptr, *d_lift_ve = nullptr;  // [term][n_h], [term][n_e]
    double lift_amp[8] = {}, lift_omega[8] = {}, lift_phase[8] = {};
    std::vector<double> lift_ve_host;  // v_e of every term (the initial Hodge)
    // last stable steps computed by kmx_cfl / kmx_cfl_scheme1 for the current
    // materials (0: not computed); steps with a larger |dt| are refused
    double dt_cfl = 0.0, dt_cfl1 = 0.0;
    int64_t frag_pre_len = 0;          // doubles in d_frag_pre (fixed by p and N)
    // optional per-kernel timing with HIP events (kmx_profile_begin/end)
    bool prof_on = false;
    unsigned prof_mask = ~0u;          // kinds bracketed with events (bit k: kind k)
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_kind;
    int prof_used = 0;
};
