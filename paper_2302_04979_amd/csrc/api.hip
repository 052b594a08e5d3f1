// C-ABI of kronmaxwell: set-up of a space and the stream-ordered leapfrog.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <unordered_set>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "kmx_internal.hpp"
#include "setup.hpp"

using namespace kmx;

// Working fields of kmx_probe_forward_noalloc (e, then h; KMX_NOALLOC_FIELD_MAX
// doubles each) in a fixed device array: every GPU the library runs on holds
// its own copy until the process ends.  Host code reaches it only through the
// per-device address from hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) double scratch[2 * KMX_NOALLOC_FIELD_MAX];

namespace {

thread_local std::string g_err;

// Spaces that exist, so that destroying a graph after its space is harmless.
std::mutex g_spaces_mu;
std::unordered_set<const kmx_space*> g_spaces;


kmx_status fail(kmx_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

// Device address of `scratch` per HIP device, resolved once per device by
// the first kmx_create_space on it (that device current).
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;

kmx_status resolve_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0) return fail(KMX_E_DEVICE, "bad device");
    if (size_t(dev) >= g_scratch_ptr.size()) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
    if (g_scratch_ptr[dev]) return KMX_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(KMX_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
    return KMX_OK;
}

double* scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return dev >= 0 && size_t(dev) < g_scratch_ptr.size() ? g_scratch_ptr[dev] : nullptr;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(KMX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

#define CHECK_LAUNCH()                                                                       \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess) return fail(KMX_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

// factor-set ids beyond the four pairing factors: 1D Gram matrices used by the
// conjugate-gradient preconditioner of the dual 2-form mass matrix
constexpr int F_GRAM_DV = 4, F_GRAM_DD = 5, NFAC = 6;
// slots of the dense operand-order factors beyond the four inverses: the
// pairing factors G^, M^, G^T, M^T themselves
constexpr int FR_PAIR = 4;

void space_dims(const kmx_space* sp, int space, int dims[3][3], int64_t off[3]) {
    for (int c = 0; c < 3; ++c) {
        comp_dims(sp, space, c, dims[c]);
        off[c] = comp_offset(sp, space, c);
    }
}

int pair_fac(int which_K1, int transpose, int c, int a) {
    if (which_K1) return transpose ? (a == c ? F_MT : F_GT) : (a == c ? F_M : F_G);
    return transpose ? (a == c ? F_G : F_M) : (a == c ? F_GT : F_MT);
}

void fill_fac(const kmx_space* sp, const double** fac, int64_t fac_off[8]) {
    *fac = sp->d_fac;
    for (int k = 0; k < 8; ++k) fac_off[k] = 0;
    for (int k = 0; k < NFAC; ++k) fac_off[k] = sp->fac_off[k];
}

// Kernel kinds reported by kmx_profile_end.
enum { PK_MASS_B = 0, PK_MASS_D = 1, PK_XY = 2, PK_Z = 3, PK_CURL = 4, PK_ENERGY = 5, PK_GATHER = 6, PK_SEP = 7,
       PK_MODE = 8, PK_DENSE = 9, PK_MASS_1 = 10, PK_VEC = 11 };

// Brackets one launch with events when profiling is on.  `by_launch`: the
// launcher takes the two events (start(), stop()) and hands them to
// hipExtLaunchKernelGGL, which stamps them when the kernel itself starts and
// ends, instead of recording them around the launch.
struct ProfScope {
    kmx_space* sp;
    hipStream_t s;
    int slot = -1;
    bool by_launch;
    ProfScope(kmx_space* sp_, hipStream_t s_, int kind, bool by_launch_ = false)
        : sp(sp_), s(s_), by_launch(by_launch_) {
        if (sp->prof_on && ((sp->prof_mask >> kind) & 1u) && sp->prof_used + 2 <= int(sp->prof_ev.size())) {
            slot = sp->prof_used;
            sp->prof_used += 2;
            sp->prof_kind[slot / 2] = kind;
            if (!by_launch) (void)hipEventRecord(sp->prof_ev[slot], s);
        }
    }
    hipEvent_t start() const { return slot >= 0 ? sp->prof_ev[slot] : nullptr; }
    hipEvent_t stop() const { return slot >= 0 ? sp->prof_ev[slot + 1] : nullptr; }
    ~ProfScope() {
        if (slot >= 0 && !by_launch) (void)hipEventRecord(sp->prof_ev[slot + 1], s);
    }
};

// y (patches) = M x or M D x for one or more batch members
void run_mass(kmx_space* sp, int space, bool curl, const double* src, int64_t src_stride, int batch,
              hipStream_t s, double* track = nullptr, int64_t track_stride = 0, double track_alpha = 0.0) {
    MassArgs a{};
    a.track = curl ? track : nullptr;
    a.track_stride = track_stride;
    a.track_alpha = track_alpha;
    space_dims(sp, space, a.track_dims, a.track_comp_off);
    a.src = src;
    a.src_stride = src_stride;
    a.patch = sp->d_patch;
    a.patch_stride = sp->patch_per_field;
    a.metric = sp->d_metric;
    a.metric_mode = sp->metric_mode;
    a.amp = sp->map.kind == 1 ? sp->map.amplitude : 0.0;
    a.axis_tab = sp->d_axis_tab;
    // 2-forms read 1/mu (B) or 1/eps (D); the 1-form masses of the first
    // scheme read eps (E) or mu (H) and their own metric factor
    a.inv_gamma = space == SP_B ? sp->d_inv_mu : space == SP_D ? sp->d_inv_eps : space == SP_E ? sp->d_eps : sp->d_mu;
    if (space == SP_E || space == SP_H) a.metric = sp->d_metric1;
    a.tab = sp->d_tab;
    for (int k = 0; k < 4; ++k) a.tab_off[k] = sp->tab_off[k];
    a.ntile = sp->ntile;
    a.npad = sp->npad;
    a.n0 = sp->n0;
    a.n1 = sp->n1;
    const int src_space = curl ? (space == SP_B ? SP_E : SP_H) : space;
    space_dims(sp, src_space, a.src_dims, a.src_comp_off);
    patch_size(sp->p, space, sp->ntile, a.patch_comp_off);
    a.waves4 = sp->mass_waves4;
    ProfScope ps(sp, s, space == SP_B ? PK_MASS_B : space == SP_D ? PK_MASS_D : PK_MASS_1, true);
    a.prof_start = ps.start();
    a.prof_stop = ps.stop();
    launch_mass(sp->p, space, curl, a, batch, s);
}

// out = (accumulate ? out : 0) + alpha * op(y), y gathered from the patches
// (from_patch) or read from `in`; op = K^{-1} (solve = 1), K (solve = 2, the
// banded pairing apply) or the identity (solve = 0, plain gather of the mass
// output).
// acc (optional, with from_patch): acc += acc_alpha * (the gathered field),
// acc with the layout of `out` and member stride acc_stride.
void run_solve(kmx_space* sp, int which_K1, int transpose, int from_patch, int gather_space, const double* in,
               int64_t in_stride, double* out, int64_t out_stride, double alpha, int accumulate, int batch,
               const kmx_source* J, double t_src, int solve, hipStream_t s, const int* fac_override = nullptr,
               const double* t_dev = nullptr, double* acc = nullptr, int64_t acc_stride = 0,
               double acc_alpha = 0.0) {
    const int64_t nfield = std::max(sp->n_e, sp->n_h);
    const int layout = which_K1 ? SP_D : SP_B;  // dims of K1 (= e, d) or K~1 (= h, b) vectors
    if (from_patch) {
        // sum the overlapping tile patches of the mass apply into a field
        GatherArgs g{};
        g.patch = sp->d_patch;
        g.patch_stride = sp->patch_per_field;
        patch_size(sp->p, gather_space == SP_B ? SP_B : SP_D, sp->ntile, g.patch_comp_off);
        space_dims(sp, layout, g.dims, g.comp_off);
        g.ntile = sp->ntile;
        const bool direct = solve == 0 && !accumulate && alpha == 1.0 && !J;
        g.out = direct ? out : sp->d_tmp2;
        g.out_stride = direct ? out_stride : nfield;
        g.acc = acc;
        g.acc_stride = acc_stride;
        g.acc_alpha = acc_alpha;
        {
            ProfScope ps(sp, s, PK_GATHER);
            launch_gather(sp->p, gather_space == SP_B ? SP_B : SP_D, g, which_K1 ? sp->n_e : sp->n_h, batch, s);
        }
        if (direct) return;
        in = sp->d_tmp2;
        in_stride = nfield;
    }
    XYArgs a{};
    a.in = in;
    a.in_stride = in_stride;
    a.out = sp->d_tmp;
    a.out_stride = nfield;
    space_dims(sp, layout, a.dims, a.comp_off);
    fill_fac(sp, &a.fac, a.fac_off);
    for (int c = 0; c < 3; ++c)
        for (int ax = 0; ax < 3; ++ax)
            a.fac_id[c][ax] = fac_override ? fac_override[c * 3 + ax] : pair_fac(which_K1, transpose, c, ax);
    a.n_src = 0;
    if (J) {
        a.src_entries = J->d_entries;
        a.src_prof = J->d_prof;
        a.src_off = reinterpret_cast<const int*>(J->d_prof + 4 * J->n);
        a.n_src = J->n;
        a.entries_per = J->entries_per;
        a.t_src = t_src;
        a.t_dev = t_dev;
    }
    a.solve = solve;
    {
        ProfScope ps(sp, s, PK_XY);
        launch_xy(sp->p, a, batch, s);
    }

    ZArgs z{};
    z.in = sp->d_tmp;
    z.in_stride = nfield;
    z.out = out;
    z.out_stride = out_stride;
    for (int c = 0; c < 3; ++c) {
        z.comp_off[c] = a.comp_off[c];
        for (int k = 0; k < 3; ++k) z.dims[c][k] = a.dims[c][k];
        z.fac_id[c] = a.fac_id[c][2];
    }
    fill_fac(sp, &z.fac, z.fac_off);
    z.alpha = alpha;
    z.accumulate = accumulate;
    z.solve = solve;
    ProfScope ps(sp, s, PK_Z);
    launch_z(sp->p, z, batch, s);
}

void run_curl(kmx_space* sp, int primal, const double* in, int64_t in_stride, double* out, int64_t out_stride,
              double alpha, double beta, int batch, hipStream_t s) {
    CurlArgs a{};
    a.in = in;
    a.in_stride = in_stride;
    a.out = out;
    a.out_stride = out_stride;
    a.alpha = alpha;
    a.beta = beta;
    a.primal = primal;
    space_dims(sp, primal ? SP_E : SP_H, a.in_dims, a.in_comp_off);
    space_dims(sp, primal ? SP_B : SP_D, a.out_dims, a.out_comp_off);
    ProfScope ps(sp, s, PK_CURL);
    launch_curl(a, primal ? sp->n_h : sp->n_e, batch, s);
}

// out += alpha * (D^1)^T y (primal: X^2_{h,0} -> X^1_{h,0}) or (D~^1)^T y (X~^2 -> X~^1)
void run_curlT(kmx_space* sp, int primal, const double* y, double* out, double alpha, hipStream_t s) {
    CurlArgs a{};
    a.in = y;
    a.out = out;
    a.alpha = alpha;
    a.beta = 1.0;
    a.primal = primal;
    space_dims(sp, primal ? SP_B : SP_D, a.in_dims, a.in_comp_off);
    space_dims(sp, primal ? SP_E : SP_H, a.out_dims, a.out_comp_off);
    launch_curlT(a, primal ? sp->n_e : sp->n_h, 1, s);
}

// blocks of the dot-product and CG reductions (per batch member)
int energy_blocks(const kmx_space* sp) {
    const int64_t n = std::max(sp->n_e, sp->n_h);
    return int(std::min<int64_t>(1024, (n + 255) / 256));
}

void run_energy(kmx_space* sp, const double* E, const double* H, double dt, int batch, double* out,
                int64_t out_stride, hipStream_t s) {
    ProfScope ps(sp, s, PK_ENERGY);
    EnergyFusedArgs a{};
    a.E = E;
    a.H = H;
    a.n_e = sp->n_e;
    a.n_h = sp->n_h;
    space_dims(sp, SP_E, a.e_dims, a.e_comp_off);
    space_dims(sp, SP_B, a.h_dims, a.h_comp_off);
    fill_fac(sp, &a.fac, a.fac_off);
    for (int c = 0; c < 3; ++c)
        for (int ax = 0; ax < 3; ++ax) {
            a.fac_id[0][c][ax] = pair_fac(1, 0, c, ax);
            a.fac_id[1][c][ax] = pair_fac(0, 0, c, ax);
        }
    a.nb[0] = energy_fused_blocks(a.e_dims, a.cb[0]);
    a.nb[1] = energy_fused_blocks(a.h_dims, a.cb[1]);
    a.partial = sp->d_red;
    launch_energy_fused(sp->p, a, batch, s);
    launch_energy_final(sp->d_red, a.nb[0] + a.nb[1], dt, batch, out, out_stride, s);
}

// Per-step energy of tracked states from the kept images w_e = K1 e and
// w_h = K~1 h (updated by the substeps) and the fields themselves.
// Step n writes its partials to half n % 2 of the reduction buffer, and its
// launch finishes step n - 1's energy from the other half (out[-batch..-1]);
// finish_energy_dots sums the last step's.
static double* energy_half(kmx_space* sp, int n, int batch) {
    return sp->d_red + int64_t(n & 1) * batch * ENERGY_DOT_WORKERS * 3;
}

void run_energy_dots(kmx_space* sp, const double* E, const double* H, double dt, int batch, int n, double* out,
                     hipStream_t s) {
    ProfScope ps(sp, s, PK_ENERGY);
    EnergyDotsArgs a{};
    a.E = E;
    a.H = H;
    a.we = sp->d_we;
    a.wh = sp->d_wh;
    a.n_e = sp->n_e;
    a.n_h = sp->n_h;
    space_dims(sp, SP_E, a.e_dims, a.e_comp_off);
    space_dims(sp, SP_B, a.h_dims, a.h_comp_off);
    a.partial = energy_half(sp, n, batch);
    if (n > 0) {
        a.prev_partial = energy_half(sp, n - 1, batch);
        a.prev_out = out - batch;
        a.prev_dt = dt;
    }
    launch_energy_dots(a, batch, s);
}

void finish_energy_dots(kmx_space* sp, double dt, int batch, int n, double* out, hipStream_t s) {
    ProfScope ps(sp, s, PK_ENERGY);
    launch_energy_final(energy_half(sp, n, batch), ENERGY_DOT_WORKERS, dt, batch, out, 1, s);
}

// The forward model of the probe misfit and its adjoint run the tiled plan,
// whose operators the reverse sweep transposes (a separable plan, chosen for
// uniform materials, cannot serve per-element eps); the space's plan is
// restored when the call returns.
struct TiledPlanScope {
    kmx_space* sp;
    int saved;
    explicit TiledPlanScope(kmx_space* s) : sp(s), saved(s->plan_kind) {
        if (saved == KMX_PLAN_SEPARABLE || saved == KMX_PLAN_SEPARABLE_FUSED) sp->plan_kind = KMX_PLAN_TILED;
    }
    ~TiledPlanScope() { sp->plan_kind = saved; }
};

LiftTerms lift_terms(const kmx_space* sp) {
    LiftTerms T{};
    T.n = sp->lift_n;
    for (int j = 0; j < sp->lift_n; ++j) {
        T.amp[j] = sp->lift_amp[j];
        T.omega[j] = sp->lift_omega[j];
        T.phase[j] = sp->lift_phase[j];
    }
    return T;
}

kmx_status upload(double** dst, const std::vector<double>& v) {
    if (hipMalloc(dst, std::max<size_t>(v.size(), 1) * sizeof(double)) != hipSuccess)
        return fail(KMX_E_OOM, "device allocation failed");
    if (!v.empty()) HIP_TRY(hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    return KMX_OK;
}

kmx_status upload_materials(kmx_space* sp) {
    const int N = sp->N, P = sp->npad;
    for (int which = 0; which < 2; ++which) {
        const std::vector<double>& h = which ? sp->inv_mu_host : sp->inv_eps_host;
        std::vector<double> pad(size_t(P) * P * P, 0.0);
        for (int z = 0; z < N; ++z)
            for (int y = 0; y < N; ++y)
                for (int x = 0; x < N; ++x)
                    pad[(size_t(z) * P + y) * P + x] = h[(size_t(z) * N + y) * N + x];
        double* d = which ? sp->d_inv_mu : sp->d_inv_eps;
        HIP_TRY(hipMemcpy(d, pad.data(), pad.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return KMX_OK;
}

// Inverse of a dense n x n matrix (row-major) by Gauss-Jordan elimination with
// partial pivoting, FP64.
std::vector<double> dense_inverse(const std::vector<double>& A, int n) {
    std::vector<double> a(A), inv(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::abs(a[size_t(i) * n + k]) > std::abs(a[size_t(piv) * n + k])) piv = i;
        if (a[size_t(piv) * n + k] == 0.0) throw std::runtime_error("singular pairing factor");
        if (piv != k)
            for (int j = 0; j < n; ++j) {
                std::swap(a[size_t(k) * n + j], a[size_t(piv) * n + j]);
                std::swap(inv[size_t(k) * n + j], inv[size_t(piv) * n + j]);
            }
        const double d = 1.0 / a[size_t(k) * n + k];
        for (int j = 0; j < n; ++j) {
            a[size_t(k) * n + j] *= d;
            inv[size_t(k) * n + j] *= d;
        }
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            const double f = a[size_t(i) * n + k];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                a[size_t(i) * n + j] -= f * a[size_t(k) * n + j];
                inv[size_t(i) * n + j] -= f * inv[size_t(k) * n + j];
            }
        }
    }
    return inv;
}

// whether eps and mu are the same in every element (a separable space needs both)
void note_uniform(kmx_space* sp) {
    sp->uniform_eps = sp->uniform_mu = true;
    for (size_t i = 1; i < sp->inv_eps_host.size(); ++i) {
        if (sp->inv_eps_host[i] != sp->inv_eps_host[0]) sp->uniform_eps = false;
        if (sp->inv_mu_host[i] != sp->inv_mu_host[0]) sp->uniform_mu = false;
    }
    sp->eps_value = sp->inv_eps_host.empty() ? 1.0 : sp->inv_eps_host[0];
    sp->mu_value = sp->inv_mu_host.empty() ? 1.0 : sp->inv_mu_host[0];
}

std::vector<double> gram(const Tables& tb, int tag) {
    const int n = (tag == PV || tag == DD) ? tb.n0 : tb.n1;
    const int K = tag_support(tb.p, tag);
    std::vector<double> G(size_t(n) * n, 0.0);
    for (int e = 0; e < tb.N; ++e)
        for (int q = 0; q < tb.nq; ++q) {
            const double* v = &tb.tab[tag][(e * tb.nq + q) * K];
            const double w = tb.wq[e * tb.nq + q];
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) {
                    const int gi = e + i + tag_offset(tag), gj = e + j + tag_offset(tag);
                    if (gi < 0 || gj < 0 || gi >= n || gj >= n) continue;
                    G[size_t(gi) * n + gj] += w * v[i] * v[j];
                }
        }
    return G;
}

}  // namespace

namespace kmx {
// Error reporting for the entry points of other sources (last error message).
kmx_status report_error(kmx_status st, const std::string& msg) { return fail(st, msg); }
// The dense inverse of a 1D pairing factor for other sources (Gauss-Jordan, FP64).
std::vector<double> pairing_inverse(const std::vector<double>& A, int n) { return dense_inverse(A, n); }
}  // namespace kmx

extern "C" {

const char* kmx_last_error(void) { return g_err.c_str(); }

kmx_status kmx_create_space(int p, int n_elem, const kmx_map* map, int precision, int max_batch,
                            kmx_space** out) {
    if (!out) return fail(KMX_E_ARG, "out is NULL");
    *out = nullptr;
    if (p < 2 || p > 4) return fail(KMX_E_ARG, "degree p must be 2, 3 or 4");
    // one xy-plane of a component ((N+p-1)^2 doubles) plus two factor sets must
    // fit the 64 KiB of dynamic LDS the solve kernel requests
    if (n_elem < 1 || n_elem > 72) return fail(KMX_E_ARG, "n_elem must be in 1..72");
    if (max_batch < 1) return fail(KMX_E_ARG, "max_batch must be >= 1");
    const int prec = precision & 0xF;
    const bool force_stored = (precision & KMX_STORED_METRIC) != 0;
    if (prec != KMX_FP64 && prec != KMX_MIXED) return fail(KMX_E_ARG, "precision must be KMX_FP64 or KMX_MIXED");
    if (precision & ~(0xF | KMX_STORED_METRIC)) return fail(KMX_E_ARG, "unknown precision flag");
    if (map && (map->kind < 0 || map->kind > 2)) return fail(KMX_E_ARG, "unknown map kind");
    if (map && map->kind == 2 && !map->dF_qp) return fail(KMX_E_ARG, "map kind 2 needs dF_qp");
    kmx_space* sp = new kmx_space();
    try {
        sp->p = p;
        sp->N = n_elem;
        sp->nq = p + 1;
        sp->n0 = n_elem + p - 2;
        sp->n1 = n_elem + p - 1;
        sp->ntile = (n_elem + TILE - 1) / TILE;
        sp->npad = sp->ntile * TILE;
        sp->max_batch = max_batch;
        sp->precision = prec;
        sp->n_e = 3LL * sp->n1 * sp->n0 * sp->n0;
        sp->n_h = 3LL * sp->n0 * sp->n1 * sp->n1;
        sp->n_qp = int64_t(n_elem) * n_elem * n_elem * sp->nq * sp->nq * sp->nq;
        sp->map = map ? *map : kmx_map{0, 0.0, nullptr};
        if (sp->map.kind == 2) {
            sp->dF_user.assign(map->dF_qp, map->dF_qp + 9 * sp->n_qp);
            sp->map.dF_qp = nullptr;
        }
        build_tables(sp->tb, p, n_elem);
        const size_t ne3 = size_t(n_elem) * n_elem * n_elem;
        sp->inv_eps_host.assign(ne3, 1.0);
        sp->inv_mu_host.assign(ne3, 1.0);
        sp->metric_mode = (sp->map.kind == 2 || force_stored) ? 0 : 1;
        std::vector<double> metric;
        kmx_status st = build_metric(sp, sp->metric_mode == 0 ? &metric : nullptr);
        if (st != KMX_OK) {
            delete sp;
            return fail(st, "det DF <= 0 at a quadrature point: the map is not admissible");
        }
        // device data
        if (sp->metric_mode == 0) {
            if ((st = upload(&sp->d_metric, metric)) != KMX_OK) { kmx_destroy_space(sp); return st; }
            std::vector<double>().swap(metric);
        }
        {
            const int64_t npq = int64_t(sp->npad) * sp->nq, nq_all = int64_t(n_elem) * sp->nq;
            std::vector<double> at(3 * npq, 0.0);
            for (int64_t i = 0; i < nq_all; ++i) {
                at[i] = std::sin(M_PI * sp->tb.xq[i]);
                at[npq + i] = std::cos(M_PI * sp->tb.xq[i]);
                at[2 * npq + i] = sp->tb.wq[i];
            }
            if ((st = upload(&sp->d_axis_tab, at)) != KMX_OK) { kmx_destroy_space(sp); return st; }
        }
        std::vector<double> tabs;
        for (int t = 0; t < 4; ++t) {
            sp->tab_off[t] = int64_t(tabs.size());
            tabs.insert(tabs.end(), sp->tb.tab[t].begin(), sp->tb.tab[t].end());
        }
        if ((st = upload(&sp->d_tab, tabs)) != KMX_OK) { kmx_destroy_space(sp); return st; }
        std::vector<double> facs;
        BandLU sets[NFAC] = {sp->tb.lu[F_G], sp->tb.lu[F_M], sp->tb.lu[F_GT], sp->tb.lu[F_MT],
                             band_lu(gram(sp->tb, DV), sp->n1, p - 1), band_lu(gram(sp->tb, DD), sp->n0, p - 1)};
        for (int k = 0; k < NFAC; ++k) {
            sp->fac_off[k] = int64_t(facs.size());
            const BandLU& f = sets[k];
            facs.insert(facs.end(), f.L.begin(), f.L.end());
            facs.insert(facs.end(), f.U.begin(), f.U.end());
            facs.insert(facs.end(), f.dinv.begin(), f.dinv.end());
            facs.insert(facs.end(), f.band.begin(), f.band.end());
        }
        if ((st = upload(&sp->d_fac, facs)) != KMX_OK) { kmx_destroy_space(sp); return st; }
        {
            // 1D Gram matrices of the four tags as bands of half width p (the
            // separable plan's Hodge factors)
            std::vector<double> gb;
            const int B = 2 * p + 1;
            for (int t = 0; t < 4; ++t) {
                sp->gram_off[t] = int64_t(gb.size());
                const int n = (t == PV || t == DD) ? sp->n0 : sp->n1;
                const std::vector<double> G = gram(sp->tb, t);
                for (int i = 0; i < n; ++i)
                    for (int k = 0; k < B; ++k) {
                        const int j = i - p + k;
                        gb.push_back(j >= 0 && j < n ? G[size_t(i) * n + j] : 0.0);
                    }
            }
            if ((st = upload(&sp->d_gram, gb)) != KMX_OK) { kmx_destroy_space(sp); return st; }
            int dev = 0;
            HIP_TRY(hipGetDevice(&dev));
            sp->device = dev;
            if ((st = resolve_scratch(dev)) != KMX_OK) { kmx_destroy_space(sp); return st; }
            HIP_TRY(hipDeviceGetAttribute(&sp->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            int ed[3][3], hd[3][3];
            int64_t o[3];
            space_dims(sp, SP_E, ed, o);
            space_dims(sp, SP_H, hd, o);
            const size_t shm = sep_lds_bytes(ed, hd);
            const int lmax = sep_line_max(std::max(sp->n0, sp->n1));
            if (lmax > 0 && shm <= size_t(sp->max_lds)) HIP_TRY(sep_prepare(p, lmax, shm));
        }
        if (std::max(sp->n0, sp->n1) <= DENSE_NMAX) {
            // dense FP64 inverses of G^, M^, G^T, M^T for the tiled-dense
            // plan, in the matrix cores' operand order
            std::vector<double> frag;
            auto add_frag = [&](int slot, const std::vector<double>& B, int n) {
                sp->frag64_off[slot] = int64_t(frag.size());
                frag.resize(frag.size() + size_t(dense_frag_doubles(n)));
                dense_fragments(B.data(), n, frag.data() + sp->frag64_off[slot]);
            };
            for (int k = 0; k < 4; ++k) {
                const int n = (k == F_G || k == F_GT) ? sp->n0 : sp->n1;
                const std::vector<double>& A = (k == F_G || k == F_GT) ? sp->tb.G : sp->tb.M;
                const std::vector<double> Ai = dense_inverse(A, n);
                std::vector<double> B(size_t(n) * n), Bf(size_t(n) * n);
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        const bool tr = k == F_GT || k == F_MT;
                        B[size_t(i) * n + j] = tr ? Ai[size_t(j) * n + i] : Ai[size_t(i) * n + j];
                        Bf[size_t(i) * n + j] = tr ? A[size_t(j) * n + i] : A[size_t(i) * n + j];
                    }
                add_frag(k, B, n);
                add_frag(FR_PAIR + k, Bf, n);
            }
            if ((st = upload(&sp->d_frag64, frag)) != KMX_OK) { kmx_destroy_space(sp); return st; }
            int db[3][3], dd[3][3];
            int64_t o[3];
            space_dims(sp, SP_B, db, o);
            space_dims(sp, SP_D, dd, o);
            const size_t shm = std::max(dense_lds_bytes(db), dense_lds_bytes(dd));
            if (shm <= size_t(sp->max_lds)) {
                HIP_TRY(dense_prepare(shm));
                sp->dense_ok = 1;
            }
        }
        if (prec == KMX_MIXED) {
            if (std::max(sp->n0, sp->n1) > mode_line_max()) {
                kmx_destroy_space(sp);
                return fail(KMX_E_ARG, "mixed precision supports lines of at most 80 entries");
            }
            // dense inverses of G^, M^, G^T, M^T in FP64, rounded to FP32
            std::vector<float> inv;
            const std::vector<double>* mats[2] = {&sp->tb.G, &sp->tb.M};
            for (int k = 0; k < 4; ++k) {
                const int n = (k == F_G || k == F_GT) ? sp->n0 : sp->n1;
                const std::vector<double>& A = *mats[(k == F_G || k == F_GT) ? 0 : 1];
                const std::vector<double> Ai = dense_inverse(A, n);
                sp->inv32_off[k] = int64_t(inv.size());
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j)
                        inv.push_back(float((k == F_GT || k == F_MT) ? Ai[size_t(j) * n + i] : Ai[size_t(i) * n + j]));
            }
            const int64_t nf = std::max(sp->n_e, sp->n_h) * int64_t(max_batch);
            if (hipMalloc(&sp->d_inv32, inv.size() * sizeof(float)) != hipSuccess ||
                hipMalloc(&sp->d_mx, nf * sizeof(double)) != hipSuccess ||
                hipMalloc(&sp->d_mr, nf * sizeof(double)) != hipSuccess ||
                hipMalloc(&sp->d_my, nf * sizeof(double)) != hipSuccess ||
                hipMalloc(&sp->d_m32a, nf * sizeof(float)) != hipSuccess ||
                hipMalloc(&sp->d_m32b, nf * sizeof(float)) != hipSuccess) {
                kmx_destroy_space(sp);
                return fail(KMX_E_OOM, "device allocation failed (mixed precision)");
            }
            HIP_TRY(hipMemcpy(sp->d_inv32, inv.data(), inv.size() * sizeof(float), hipMemcpyHostToDevice));
        }
        const size_t npad3 = size_t(sp->npad) * sp->npad * sp->npad;
        if (hipMalloc(&sp->d_inv_eps, npad3 * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_inv_mu, npad3 * sizeof(double)) != hipSuccess) {
            kmx_destroy_space(sp);
            return fail(KMX_E_OOM, "device allocation failed (materials)");
        }
        if ((st = upload_materials(sp)) != KMX_OK) { kmx_destroy_space(sp); return st; }
        int64_t off[3];
        sp->patch_per_field = 0;
        for (int space = 0; space < 4; ++space)
            sp->patch_per_field = std::max(sp->patch_per_field, patch_size(p, space, sp->ntile, off));
        const int64_t nfield = std::max(sp->n_e, sp->n_h);
        {
            // reduction partials: the CG and dot kernels use up to 1024 blocks per
            // member, the per-step energy dots two halves of ENERGY_DOT_BLOCKS,
            // the fused energy kernel one per (component, plane, row block)
            int ed[3][3], hd[3][3], cb[3];
            int64_t o[3];
            space_dims(sp, SP_E, ed, o);
            space_dims(sp, SP_B, hd, o);
            const int64_t nbe = energy_fused_blocks(ed, cb) + energy_fused_blocks(hd, cb);
            sp->red_len = int64_t(max_batch) * std::max<int64_t>(std::max(1024, 2 * ENERGY_DOT_BLOCKS), nbe) * 3 + 64;
        }
        if (hipMalloc(&sp->d_patch, size_t(sp->patch_per_field) * max_batch * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_tmp, size_t(nfield) * max_batch * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_tmp2, size_t(nfield) * max_batch * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_we, size_t(sp->n_e) * max_batch * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_wh, size_t(sp->n_h) * max_batch * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_red, size_t(sp->red_len) * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_scal, size_t(64 + 2 * max_batch) * sizeof(double)) != hipSuccess ||
            hipMalloc(&sp->d_time, sizeof(double)) != hipSuccess) {
            kmx_destroy_space(sp);
            return fail(KMX_E_OOM, "device allocation failed (scratch)");
        }
    } catch (const std::exception& ex) {
        kmx_destroy_space(sp);
        return fail(KMX_E_ARG, std::string("set-up failed: ") + ex.what());
    }
    {
        std::lock_guard<std::mutex> lk(g_spaces_mu);
        g_spaces.insert(sp);
    }
    *out = sp;
    return KMX_OK;
}

kmx_status kmx_profile_begin(kmx_space* sp, int capacity) {
    if (!sp || capacity < 1) return fail(KMX_E_ARG, "bad argument");
    if (sp->prof_on) return fail(KMX_E_STATE, "profiling already on");
    sp->prof_ev.assign(2 * size_t(capacity), nullptr);
    sp->prof_kind.assign(capacity, -1);
    for (auto& e : sp->prof_ev) HIP_TRY(hipEventCreate(&e));
    sp->prof_used = 0;
    sp->prof_on = true;
    return KMX_OK;
}

kmx_status kmx_profile_select(kmx_space* sp, unsigned mask) {
    if (!sp) return fail(KMX_E_ARG, "space is NULL");
    if (mask == 0 || (mask >> KMX_PROFILE_KINDS) != 0) return fail(KMX_E_ARG, "mask must name kinds 0..KMX_PROFILE_KINDS-1");
    sp->prof_mask = mask;
    return KMX_OK;
}

kmx_status kmx_profile_end(kmx_space* sp, double* ms_total, int* launches) {
    if (!sp || !ms_total || !launches) return fail(KMX_E_ARG, "bad argument");
    if (!sp->prof_on) return fail(KMX_E_STATE, "profiling is off");
    for (int k = 0; k < KMX_PROFILE_KINDS; ++k) {
        ms_total[k] = 0.0;
        launches[k] = 0;
    }
    kmx_status st = KMX_OK;
    if (sp->prof_used > 0 && hipEventSynchronize(sp->prof_ev[sp->prof_used - 1]) != hipSuccess)
        st = fail(KMX_E_DEVICE, "event synchronisation failed");
    for (int i = 0; st == KMX_OK && i < sp->prof_used / 2; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp->prof_ev[2 * i], sp->prof_ev[2 * i + 1]) != hipSuccess) {
            st = fail(KMX_E_DEVICE, "hipEventElapsedTime failed");
            break;
        }
        ms_total[sp->prof_kind[i]] += ms;
        launches[sp->prof_kind[i]] += 1;
    }
    for (auto& e : sp->prof_ev) (void)hipEventDestroy(e);
    for (auto& e : sp->s1_ev)
        if (e) (void)hipEventDestroy(e);
    if (sp->h_rr) (void)hipHostFree(sp->h_rr);
    sp->prof_ev.clear();
    sp->prof_kind.clear();
    sp->prof_used = 0;
    sp->prof_on = false;
    sp->prof_mask = ~0u;
    return st;
}

void kmx_destroy_space(kmx_space* sp) {
    if (!sp) return;
    {
        std::lock_guard<std::mutex> lk(g_spaces_mu);
        g_spaces.erase(sp);
    }
    for (auto& e : sp->prof_ev) (void)hipEventDestroy(e);
    for (auto& e : sp->s1_ev)
        if (e) (void)hipEventDestroy(e);
    if (sp->h_rr) (void)hipHostFree(sp->h_rr);
    if (sp->capture_stream) (void)hipStreamDestroy(sp->capture_stream);
    if (sp->d_time) (void)hipFree(sp->d_time);
    double* bufs[] = {sp->d_tab, sp->d_metric, sp->d_axis_tab, sp->d_inv_eps, sp->d_inv_mu, sp->d_fac,
                      sp->d_gram, sp->d_patch, sp->d_tmp, sp->d_tmp2, sp->d_we, sp->d_wh, sp->d_red, sp->d_scal};
    for (double* b : bufs)
        if (b) (void)hipFree(b);
    void* more[] = {sp->d_inv32, sp->d_mx, sp->d_mr, sp->d_my, sp->d_m32a, sp->d_m32b, sp->d_frag64,
                    sp->d_eps, sp->d_mu, sp->d_metric1, sp->d_s1, sp->d_frag_pre, sp->d_lift_vh,
                    sp->d_lift_ve};
    for (void* b : more)
        if (b) (void)hipFree(b);
    delete sp;
}

kmx_status kmx_set_materials(kmx_space* sp, const double* eps_elem, const double* mu_elem) {
    if (!sp) return fail(KMX_E_ARG, "space is NULL");
    if (sp->live_graphs > 0)
        return fail(KMX_E_STATE, "graphs of this space exist: they hold the material state they were captured "
                                 "with; destroy them before changing the materials");
    const size_t ne3 = size_t(sp->N) * sp->N * sp->N;
    std::vector<double> ie(ne3, 1.0), im(ne3, 1.0);
    for (size_t i = 0; i < ne3; ++i) {
        if (eps_elem) {
            if (!(eps_elem[i] > 0.0) || !std::isfinite(eps_elem[i]))
                return fail(KMX_E_MATERIAL, "eps must be finite and > 0");
            ie[i] = 1.0 / eps_elem[i];
        }
        if (mu_elem) {
            if (!(mu_elem[i] > 0.0) || !std::isfinite(mu_elem[i]))
                return fail(KMX_E_MATERIAL, "mu must be finite and > 0");
            im[i] = 1.0 / mu_elem[i];
        }
    }
    sp->inv_eps_host = ie;
    sp->inv_mu_host = im;
    if (eps_elem) sp->eps_host.assign(eps_elem, eps_elem + ne3);
    else sp->eps_host.clear();
    if (mu_elem) sp->mu_host.assign(mu_elem, mu_elem + ne3);
    else sp->mu_host.clear();
    sp->s1_ready = 0;
    sp->dt_cfl = sp->dt_cfl1 = 0.0;  // the stable steps change with the materials
    sp->lift_n = 0;                  // the lifting's v_h depends on mu: set it again
    note_uniform(sp);
    return upload_materials(sp);
}

kmx_status kmx_sizes_full(const kmx_space* sp, int64_t* n_ef) {
    if (!sp || !n_ef) return fail(KMX_E_ARG, "NULL argument");
    *n_ef = full_size(sp, 1);
    return KMX_OK;
}

kmx_status kmx_lift_boundary(kmx_space* sp, const double* Eh_faces, double* eb_full, int* iters) {
    if (!sp || !Eh_faces || !eb_full) return fail(KMX_E_ARG, "NULL argument");
    const int64_t nq = int64_t(sp->N) * sp->nq;
    for (int64_t i = 0; i < 6 * nq * nq * 3; ++i)
        if (!std::isfinite(Eh_faces[i])) return fail(KMX_E_ARG, "face data not finite");
    const int it = boundary_fit(sp, Eh_faces, eb_full, 1e-14, 5000);
    if (iters) *iters = it;
    if (it < 0) return fail(KMX_E_UNSTABLE, "the trace fit did not converge");
    return KMX_OK;
}

kmx_status kmx_set_lifting(kmx_space* sp, int nterms, const double* eb_full, const double* amp, const double* omega,
                           const double* phase) {
    if (!sp || nterms < 0 || nterms > KMX_LIFT_MAX) return fail(KMX_E_ARG, "nterms must be 0..8");
    if (nterms > 0 && (!eb_full || !amp || !omega || !phase)) return fail(KMX_E_ARG, "NULL argument");
    if (sp->live_graphs > 0) return fail(KMX_E_STATE, "graphs of this space exist: destroy them first");
    for (int j = 0; j < nterms; ++j)
        if (!std::isfinite(amp[j]) || !std::isfinite(omega[j]) || !std::isfinite(phase[j]))
            return fail(KMX_E_ARG, "time profile not finite");
    sp->lift_n = 0;
    if (nterms == 0) return KMX_OK;
    const int64_t nf = full_size(sp, 1), nh = sp->n_h, ne = sp->n_e;
    for (int64_t i = 0; i < nterms * nf; ++i)
        if (!std::isfinite(eb_full[i])) return fail(KMX_E_ARG, "boundary coefficients not finite");
    std::vector<double> vh_all(size_t(nterms) * nh), ve_all(size_t(nterms) * ne);
    for (int j = 0; j < nterms; ++j) {
        std::vector<double> vh, ve;
        lifting_vectors(sp, eb_full + int64_t(j) * nf, vh, ve);
        std::copy(vh.begin(), vh.end(), vh_all.begin() + int64_t(j) * nh);
        std::copy(ve.begin(), ve.end(), ve_all.begin() + int64_t(j) * ne);
    }
    if (sp->d_lift_vh) { hipFree(sp->d_lift_vh); sp->d_lift_vh = nullptr; }
    if (sp->d_lift_ve) { hipFree(sp->d_lift_ve); sp->d_lift_ve = nullptr; }
    kmx_status st;
    if ((st = upload(&sp->d_lift_vh, vh_all)) != KMX_OK) return st;
    if ((st = upload(&sp->d_lift_ve, ve_all)) != KMX_OK) return st;
    sp->lift_ve_host.swap(ve_all);
    for (int j = 0; j < nterms; ++j) {
        sp->lift_amp[j] = amp[j];
        sp->lift_omega[j] = omega[j];
        sp->lift_phase[j] = phase[j];
    }
    sp->lift_n = nterms;
    return KMX_OK;
}

kmx_status kmx_sizes(const kmx_space* sp, int64_t* n_e, int64_t* n_h, int64_t* n_qp) {
    if (!sp) return fail(KMX_E_ARG, "space is NULL");
    if (n_e) *n_e = sp->n_e;
    if (n_h) *n_h = sp->n_h;
    if (n_qp) *n_qp = sp->n_qp;
    return KMX_OK;
}

kmx_status kmx_quad_points(const kmx_space* sp, double* xyz_host) {
    if (!sp || !xyz_host) return fail(KMX_E_ARG, "NULL argument");
    quad_points(sp, xyz_host);
    return KMX_OK;
}

kmx_status kmx_project_E(kmx_space* sp, const double* E_qp_host, double* e_dev, void* stream) {
    if (!sp || !E_qp_host || !e_dev) return fail(KMX_E_ARG, "NULL argument");
    std::vector<double> l;
    load_E(sp, E_qp_host, l);
    kron_solve_K1_host(sp, l);
    // with a lifting: (K1)_0 e = l - (K1)_b e_b(0)
    for (int j = 0; j < sp->lift_n; ++j) {
        const double g0 = sp->lift_amp[j] * std::cos(sp->lift_phase[j]);
        for (int64_t i = 0; i < sp->n_e; ++i) l[i] -= g0 * sp->lift_ve_host[size_t(j) * sp->n_e + i];
    }
    HIP_TRY(hipMemcpyAsync(e_dev, l.data(), l.size() * sizeof(double), hipMemcpyHostToDevice,
                           static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return KMX_OK;
}

kmx_status kmx_project_D(kmx_space* sp, const double* E_qp_host, double* d_dev, double tol, void* stream) {
    if (!sp || !E_qp_host || !d_dev) return fail(KMX_E_ARG, "NULL argument");
    if (!(tol > 0.0)) return fail(KMX_E_ARG, "tol must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<double> l;
    load_E(sp, E_qp_host, l);
    const int64_t n = sp->n_e;
    double *r = nullptr, *z = nullptr, *pd = nullptr, *Ap = nullptr;
    if (hipMalloc(&r, n * sizeof(double)) != hipSuccess || hipMalloc(&z, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&pd, n * sizeof(double)) != hipSuccess || hipMalloc(&Ap, n * sizeof(double)) != hipSuccess) {
        hipFree(r); hipFree(z); hipFree(pd); hipFree(Ap);
        return fail(KMX_E_OOM, "device allocation failed (CG vectors)");
    }
    kmx_status result = KMX_OK;
    const int nb = energy_blocks(sp);
    int pre[9];
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 3; ++a) pre[c * 3 + a] = (a == c) ? F_GRAM_DV : F_GRAM_DD;
    auto dot = [&](const double* x, const double* y, int slot) {
        launch_dot(x, y, n, n, 1, sp->d_red, nb, s);
        launch_sum_final(sp->d_red, nb, 1, sp->d_scal + slot, s);
    };
    auto precond = [&](const double* in, double* outv) {  // identity-map, unit-material mass inverse
        run_solve(sp, 1, 0, 0, SP_D, in, n, outv, n, 1.0, 0, 1, nullptr, 0.0, 1, s, pre);
    };
    double l2 = 0.0;
    for (double v : l) l2 += v * v;
    const double stop = tol * std::sqrt(l2);
    hipMemcpyAsync(r, l.data(), n * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemsetAsync(d_dev, 0, n * sizeof(double), s);
    precond(r, z);
    hipMemcpyAsync(pd, z, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    dot(r, z, 0);
    int it = 0;
    for (; it < 2000; ++it) {
        run_mass(sp, SP_D, false, pd, n, 1, s);
        run_solve(sp, 1, 0, 1, SP_D, nullptr, 0, Ap, n, 1.0, 0, 1, nullptr, 0.0, 0, s);
        dot(pd, Ap, 1);
        launch_cg_update(d_dev, r, pd, Ap, nullptr, n, sp->d_scal, 0, s);
        dot(r, r, 3);
        double rr = 0.0;
        hipMemcpyAsync(&rr, sp->d_scal + 3, sizeof(double), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess) { result = fail(KMX_E_DEVICE, "CG failed"); break; }
        if (!std::isfinite(rr)) { result = fail(KMX_E_UNSTABLE, "CG diverged"); break; }
        if (std::sqrt(rr) <= stop) break;
        precond(r, z);
        dot(r, z, 2);
        launch_cg_update(d_dev, r, pd, Ap, z, n, sp->d_scal, 1, s);
        hipMemcpyAsync(sp->d_scal, sp->d_scal + 2, sizeof(double), hipMemcpyDeviceToDevice, s);
    }
    if (result == KMX_OK && it >= 2000) result = fail(KMX_E_UNSTABLE, "CG did not converge");
    hipStreamSynchronize(s);
    hipFree(r); hipFree(z); hipFree(pd); hipFree(Ap);
    return result;
}

kmx_status kmx_cfl(kmx_space* sp, int max_iter, double tol, double* dt_max) {
    if (!sp || !dt_max || max_iter < 1) return fail(KMX_E_ARG, "bad argument");
    hipStream_t s = nullptr;
    const int64_t ne = sp->n_e, nh = sp->n_h;
    double *x = nullptr, *hb = nullptr;
    if (hipMalloc(&x, ne * sizeof(double)) != hipSuccess || hipMalloc(&hb, nh * sizeof(double)) != hipSuccess) {
        hipFree(x); hipFree(hb);
        return fail(KMX_E_OOM, "device allocation failed (CFL vectors)");
    }
    std::vector<double> x0(ne);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    double nrm = 0.0;
    for (int64_t i = 0; i < ne; ++i) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        x0[i] = double(st >> 11) / double(1ull << 53) - 0.5;
        nrm += x0[i] * x0[i];
    }
    for (auto& v : x0) v /= std::sqrt(nrm);
    hipMemcpy(x, x0.data(), ne * sizeof(double), hipMemcpyHostToDevice);
    const int nb = energy_blocks(sp);
    double lam = 0.0;
    kmx_status result = KMX_OK;
    for (int it = 0; it < max_iter; ++it) {
        run_mass(sp, SP_B, true, x, ne, 1, s);
        run_solve(sp, 0, 0, 1, SP_B, nullptr, 0, hb, nh, 1.0, 0, 1, nullptr, 0.0, 1, s);
        run_mass(sp, SP_D, true, hb, nh, 1, s);
        run_solve(sp, 1, 0, 1, SP_D, nullptr, 0, x, ne, 1.0, 0, 1, nullptr, 0.0, 1, s);
        launch_dot(x, x, ne, ne, 1, sp->d_red, nb, s);
        launch_sum_final(sp->d_red, nb, 1, sp->d_scal, s);
        double yy = 0.0;
        hipMemcpy(&yy, sp->d_scal, sizeof(double), hipMemcpyDeviceToHost);
        const double lam_new = std::sqrt(yy);
        if (!std::isfinite(lam_new) || lam_new <= 0.0) { result = fail(KMX_E_UNSTABLE, "power iteration failed"); break; }
        launch_axpby(x, x, ne, 1.0 / lam_new, nullptr, 0.0, s);
        const bool done = std::fabs(lam_new - lam) <= tol * lam_new;
        lam = lam_new;
        if (done) break;
    }
    hipDeviceSynchronize();
    hipFree(x);
    hipFree(hb);
    if (result != KMX_OK) return result;
    *dt_max = 2.0 / std::sqrt(lam);
    sp->dt_cfl = *dt_max;
    return KMX_OK;
}

kmx_status kmx_create_source(kmx_space* sp, int n, const double* pos, const double* moment, const double* t0,
                             const double* sigma, const double* amp, const int* batch_of, kmx_source** out) {
    if (!sp || !out || n < 1 || !pos || !moment || !t0 || !sigma || !amp) return fail(KMX_E_ARG, "bad argument");
    *out = nullptr;
    std::vector<int> order(n);
    for (int k = 0; k < n; ++k) {
        order[k] = k;
        const int b = batch_of ? batch_of[k] : 0;
        if (b < 0 || b >= sp->max_batch) return fail(KMX_E_ARG, "dipole batch index out of range");
        for (int a = 0; a < 3; ++a)
            if (!(pos[3 * k + a] >= 0.0 && pos[3 * k + a] <= 1.0)) return fail(KMX_E_ARG, "dipole position outside [0,1]^3");
        if (!(sigma[k] > 0.0)) return fail(KMX_E_ARG, "sigma must be > 0");
    }
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) {
        return (batch_of ? batch_of[i] : 0) < (batch_of ? batch_of[j] : 0);
    });
    const int per = 3 * sp->p * (sp->p - 1) * (sp->p - 1);
    std::vector<double> ent(size_t(n) * per * 5, 0.0), prof(size_t(n) * 4);
    std::vector<int> off(sp->max_batch + 1, 0);
    int bmax = 0;
    for (int r = 0; r < n; ++r) {
        const int k = order[r];
        std::vector<DipoleEntry> de;
        dipole_entries(sp, &pos[3 * k], &moment[3 * k], de);
        for (size_t e = 0; e < de.size() && int(e) < per; ++e) {
            double* q = &ent[(size_t(r) * per + e) * 5];
            q[0] = de[e].comp; q[1] = de[e].iz; q[2] = de[e].iy; q[3] = de[e].ix; q[4] = de[e].val;
        }
        for (size_t e = de.size(); int(e) < per; ++e) ent[(size_t(r) * per + e) * 5] = -1.0;  // no component
        const int b = batch_of ? batch_of[k] : 0;
        prof[4 * r] = t0[k]; prof[4 * r + 1] = sigma[k]; prof[4 * r + 2] = amp[k]; prof[4 * r + 3] = b;
        off[b + 1]++;
        bmax = std::max(bmax, b + 1);
    }
    for (int b = 0; b < sp->max_batch; ++b) off[b + 1] += off[b];
    std::vector<int> elem(n);
    std::vector<double> src_ie(n);
    for (int r = 0; r < n; ++r) {
        const int k = order[r];
        int el[3];
        for (int a = 0; a < 3; ++a)
            el[a] = std::min(std::max(int(std::floor(pos[3 * k + a] * sp->N)), 0), sp->N - 1);
        elem[r] = (el[2] * sp->N + el[1]) * sp->N + el[0];
        src_ie[r] = sp->inv_eps_host[elem[r]];
    }
    kmx_source* src = new kmx_source();
    src->sp = sp;
    src->n = n;
    src->batch_max = bmax;
    src->entries_per = per;
    // offsets are stored as ints right after the profiles
    const size_t prof_bytes = prof.size() * sizeof(double), off_bytes = off.size() * sizeof(int);
    if (hipMalloc(&src->d_entries, ent.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&src->d_prof, prof_bytes + off_bytes + 16) != hipSuccess) {
        kmx_destroy_source(src);
        return fail(KMX_E_OOM, "device allocation failed (sources)");
    }
    HIP_TRY(hipMemcpy(src->d_entries, ent.data(), ent.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(src->d_prof, prof.data(), prof_bytes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(reinterpret_cast<char*>(src->d_prof) + prof_bytes, off.data(), off_bytes, hipMemcpyHostToDevice));
    int dims[3][3];
    int64_t coff[3];
    space_dims(sp, SP_D, dims, coff);
    if (hipMalloc(&src->d_elem, n * sizeof(int)) != hipSuccess ||
        hipMalloc(&src->d_inv_eps, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&src->d_comp_off, 3 * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&src->d_dims, 9 * sizeof(int)) != hipSuccess) {
        kmx_destroy_source(src);
        return fail(KMX_E_OOM, "device allocation failed (sources)");
    }
    HIP_TRY(hipMemcpy(src->d_elem, elem.data(), n * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(src->d_inv_eps, src_ie.data(), n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(src->d_comp_off, coff, 3 * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(src->d_dims, &dims[0][0], 9 * sizeof(int), hipMemcpyHostToDevice));
    *out = src;
    return KMX_OK;
}

kmx_status kmx_create_source_pattern(kmx_space* sp, int npat, const double* pattern, int nsamples, double t0,
                                     double dt_sample, const double* series, kmx_source** out) {
    if (!sp || !out || !pattern || !series) return fail(KMX_E_ARG, "NULL argument");
    *out = nullptr;
    if (npat < 1 || npat > sp->max_batch) return fail(KMX_E_ARG, "npat must be 1..max_batch");
    if (nsamples < 2) return fail(KMX_E_ARG, "the time series needs at least two samples");
    if (!std::isfinite(t0) || !(dt_sample > 0.0) || !std::isfinite(dt_sample))
        return fail(KMX_E_ARG, "t0 must be finite and dt_sample > 0");
    const int64_t n = int64_t(npat) * sp->n_e;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(pattern[i])) return fail(KMX_E_ARG, "pattern entry not finite");
    for (int k = 0; k < nsamples; ++k)
        if (!std::isfinite(series[k])) return fail(KMX_E_ARG, "series sample not finite");
    kmx_source* src = new kmx_source();
    src->sp = sp;
    src->kind = 1;
    src->npat = npat;
    src->nsamples = nsamples;
    src->ts0 = t0;
    src->tsh = dt_sample;
    src->batch_max = npat;
    if (hipMalloc(&src->d_pattern, size_t(n) * sizeof(double)) != hipSuccess ||
        hipMalloc(&src->d_series, size_t(nsamples) * sizeof(double)) != hipSuccess) {
        kmx_destroy_source(src);
        return fail(KMX_E_OOM, "device allocation failed (source pattern)");
    }
    if (hipMemcpy(src->d_pattern, pattern, size_t(n) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(src->d_series, series, size_t(nsamples) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        kmx_destroy_source(src);
        return fail(KMX_E_DEVICE, "copy of the source pattern failed");
    }
    *out = src;
    return KMX_OK;
}

void kmx_destroy_source(kmx_source* src) {
    if (!src) return;
    if (src->d_pattern) (void)hipFree(src->d_pattern);
    if (src->d_series) (void)hipFree(src->d_series);
    if (src->d_entries) (void)hipFree(src->d_entries);
    if (src->d_prof) (void)hipFree(src->d_prof);
    if (src->d_elem) (void)hipFree(src->d_elem);
    if (src->d_inv_eps) (void)hipFree(src->d_inv_eps);
    if (src->d_comp_off) (void)hipFree(src->d_comp_off);
    if (src->d_dims) (void)hipFree(src->d_dims);
    delete src;
}

kmx_status kmx_create_probes(kmx_space* sp, int n, const double* pos, kmx_probes** out) {
    if (!sp || !pos || !out || n < 1) return fail(KMX_E_ARG, "bad argument");
    *out = nullptr;
    const Tables& tb = sp->tb;
    const int N = sp->N, p = sp->p;
    struct Ent { int row; int col; double val; };
    std::vector<Ent> ents;
    for (int k = 0; k < n; ++k) {
        const double* xh = pos + 3 * k;
        int el[3];
        for (int a = 0; a < 3; ++a) {
            if (!(xh[a] >= 0.0 && xh[a] <= 1.0)) return fail(KMX_E_ARG, "probe position outside [0,1]^3");
            el[a] = std::min(std::max(int(std::floor(xh[a] * N)), 0), N - 1);
        }
        double J[9];
        map_jacobian(sp, sp->map.kind == 2 ? (((int64_t(el[2]) * N + el[1]) * N + el[0]) * sp->nq * sp->nq * sp->nq)
                                           : -1, xh, J);
        // inverse transpose of DF: E = DF^{-T} E^ (covariant pullback of 1-forms)
        const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                           J[2] * (J[3] * J[7] - J[4] * J[6]);
        double C[9];  // cofactor matrix: DF^{-T} = C / det
        C[0] = J[4] * J[8] - J[5] * J[7]; C[1] = -(J[3] * J[8] - J[5] * J[6]); C[2] = J[3] * J[7] - J[4] * J[6];
        C[3] = -(J[1] * J[8] - J[2] * J[7]); C[4] = J[0] * J[8] - J[2] * J[6]; C[5] = -(J[0] * J[7] - J[1] * J[6]);
        C[6] = J[1] * J[5] - J[2] * J[4]; C[7] = -(J[0] * J[5] - J[2] * J[3]); C[8] = J[0] * J[4] - J[1] * J[3];
        for (int j = 0; j < 3; ++j) {
            int d[3];
            comp_dims(sp, SP_E, j, d);
            const int64_t off = comp_offset(sp, SP_E, j);
            double bv[3][8];
            int K[3], tg[3];
            for (int a = 0; a < 3; ++a) {
                tg[a] = space_tag(SP_E, j, a);
                K[a] = tag_support(p, tg[a]);
                eval_tag_on_element(tb, tg[a], el[a], xh[a], bv[a]);
            }
            for (int jz = 0; jz < K[2]; ++jz)
                for (int jy = 0; jy < K[1]; ++jy)
                    for (int jx = 0; jx < K[0]; ++jx) {
                        const int gx = el[0] + jx + tag_offset(tg[0]), gy = el[1] + jy + tag_offset(tg[1]),
                                  gz = el[2] + jz + tag_offset(tg[2]);
                        if (gx < 0 || gy < 0 || gz < 0 || gx >= d[2] || gy >= d[1] || gz >= d[0]) continue;
                        const double w = bv[2][jz] * bv[1][jy] * bv[0][jx];
                        if (w == 0.0) continue;
                        const int col = int(off + (int64_t(gz) * d[1] + gy) * d[2] + gx);
                        for (int c = 0; c < 3; ++c) ents.push_back({3 * k + c, col, C[3 * c + j] / det * w});
                    }
        }
    }
    // P in CSR (rows in order, entries in construction order)
    std::vector<int> rowptr(3 * n + 1, 0), col;
    std::vector<double> val;
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) { return a.row < b.row; });
    for (const Ent& e : ents) { rowptr[e.row + 1]++; col.push_back(e.col); val.push_back(e.val); }
    for (int r = 0; r < 3 * n; ++r) rowptr[r + 1] += rowptr[r];
    // P^T over the touched dofs
    std::vector<Ent> tents(ents);
    std::stable_sort(tents.begin(), tents.end(), [](const Ent& a, const Ent& b) {
        return a.col < b.col || (a.col == b.col && a.row < b.row);
    });
    std::vector<int> trowptr(1, 0), tcol, tidx;
    std::vector<double> tval;
    for (size_t i = 0; i < tents.size(); ++i) {
        if (i == 0 || tents[i].col != tents[i - 1].col) {
            tidx.push_back(tents[i].col);
            if (i) trowptr.push_back(int(i));
        }
        tcol.push_back(tents[i].row);
        tval.push_back(tents[i].val);
    }
    trowptr.push_back(int(tents.size()));
    kmx_probes* pr = new kmx_probes();
    pr->sp = sp;
    pr->n = n;
    pr->ntrows = int(tidx.size());
    auto up_i = [&](int** d, const std::vector<int>& v) {
        return hipMalloc(d, std::max<size_t>(v.size(), 1) * sizeof(int)) == hipSuccess &&
               (v.empty() || hipMemcpy(*d, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess);
    };
    auto up_d = [&](double** d, const std::vector<double>& v) {
        return hipMalloc(d, std::max<size_t>(v.size(), 1) * sizeof(double)) == hipSuccess &&
               (v.empty() || hipMemcpy(*d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess);
    };
    if (!up_i(&pr->d_rowptr, rowptr) || !up_i(&pr->d_col, col) || !up_d(&pr->d_val, val) ||
        !up_i(&pr->d_trowptr, trowptr) || !up_i(&pr->d_tcol, tcol) || !up_i(&pr->d_tidx, tidx) ||
        !up_d(&pr->d_tval, tval)) {
        kmx_destroy_probes(pr);
        return fail(KMX_E_OOM, "device allocation failed (probes)");
    }
    *out = pr;
    return KMX_OK;
}

void kmx_destroy_probes(kmx_probes* pr) {
    if (!pr) return;
    int* ib[] = {pr->d_rowptr, pr->d_col, pr->d_trowptr, pr->d_tcol, pr->d_tidx};
    for (int* b : ib)
        if (b) (void)hipFree(b);
    if (pr->d_val) (void)hipFree(pr->d_val);
    if (pr->d_tval) (void)hipFree(pr->d_tval);
    delete pr;
}

kmx_status kmx_probe_eval(kmx_space* sp, const kmx_probes* pr, const double* e, double* out, void* stream) {
    if (!sp || !pr || !e || !out || pr->sp != sp) return fail(KMX_E_ARG, "bad argument");
    launch_csr(pr->d_rowptr, pr->d_col, pr->d_val, e, out, nullptr, 3 * pr->n, 1.0, 0.0,
               static_cast<hipStream_t>(stream));
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_probe_forward(kmx_space* sp, const kmx_probes* pr, const kmx_source* J, double dt, int nsteps,
                             double* obs, void* stream) {
    if (!sp || !pr || !obs || nsteps < 1 || pr->sp != sp || (J && J->sp != sp)) return fail(KMX_E_ARG, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const TiledPlanScope tiled(sp);
    double *e = nullptr, *h = nullptr;
    if (hipMalloc(&e, sp->n_e * sizeof(double)) != hipSuccess || hipMalloc(&h, sp->n_h * sizeof(double)) != hipSuccess) {
        hipFree(e); hipFree(h);
        return fail(KMX_E_OOM, "device allocation failed");
    }
    hipMemsetAsync(e, 0, sp->n_e * sizeof(double), s);
    hipMemsetAsync(h, 0, sp->n_h * sizeof(double), s);
    kmx_status st = KMX_OK;
    for (int n = 0; n < nsteps && st == KMX_OK; ++n) {
        st = kmx_step(sp, e, h, J, n * dt, dt, 1, 1, 0, nullptr, stream);
        launch_csr(pr->d_rowptr, pr->d_col, pr->d_val, e, obs + int64_t(n) * 3 * pr->n, nullptr, 3 * pr->n, 1.0,
                   0.0, s);
    }
    hipStreamSynchronize(s);
    hipFree(e);
    hipFree(h);
    if (st != KMX_OK) return st;
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_probe_forward_noalloc(kmx_space* sp, const kmx_probes* pr, const kmx_source* J, double dt,
                                     int nsteps, double* obs, void* stream) {
    if (!sp || !pr || !obs || nsteps < 1 || pr->sp != sp || (J && J->sp != sp)) return fail(KMX_E_ARG, "bad argument");
    if (sp->n_e > KMX_NOALLOC_FIELD_MAX || sp->n_h > KMX_NOALLOC_FIELD_MAX)
        return fail(KMX_E_ARG, "fields larger than KMX_NOALLOC_FIELD_MAX entries: use kmx_probe_forward");
    double* base = scratch_ptr(sp->device);
    if (!base) return fail(KMX_E_STATE, "the fixed working array of this device is not resolved");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const TiledPlanScope tiled(sp);
    double* e = base;
    double* h = base + KMX_NOALLOC_FIELD_MAX;
    // the array keeps the previous call's values: start from zero fields
    launch_fill(e, sp->n_e, 0.0, s);
    launch_fill(h, sp->n_h, 0.0, s);
    kmx_status st = KMX_OK;
    for (int n = 0; n < nsteps && st == KMX_OK; ++n) {
        st = kmx_step(sp, e, h, J, n * dt, dt, 1, 1, 0, nullptr, stream);
        launch_csr(pr->d_rowptr, pr->d_col, pr->d_val, e, obs + int64_t(n) * 3 * pr->n, nullptr, 3 * pr->n, 1.0,
                   0.0, s);
    }
    if (st != KMX_OK) return st;
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_adjoint(kmx_space* sp, const kmx_probes* pr, const kmx_source* J, const double* data, double dt,
                       int nsteps, int checkpoint_every, double* loss_host, double* grad, void* stream) {
    if (!sp || !pr || !data || !loss_host || !grad || nsteps < 1 || checkpoint_every < 1 || pr->sp != sp ||
        (J && J->sp != sp))
        return fail(KMX_E_ARG, "bad argument");
    if (sp->lift_n) return fail(KMX_E_STATE, "the adjoint does not take a lifting");
    if (J && J->kind == 1) return fail(KMX_E_STATE, "the adjoint takes point dipoles only");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const TiledPlanScope tiled(sp);
    const int64_t ne = sp->n_e, nh = sp->n_h, nobs = int64_t(3) * pr->n, NS = nsteps;
    const int K = std::min(checkpoint_every, nsteps), nseg = (nsteps + K - 1) / K;
    // working memory (this call allocates; the time step itself never does)
    std::vector<double*> bufs;
    auto alloc = [&](int64_t count) -> double* {
        double* p = nullptr;
        if (hipMalloc(&p, std::max<int64_t>(count, 1) * sizeof(double)) != hipSuccess) return nullptr;
        bufs.push_back(p);
        return p;
    };
    double* ck_e = alloc(nseg * ne);
    double* ck_h = alloc(nseg * nh);
    double* seg_h = alloc(int64_t(K) * nh);
    double* e = alloc(ne);
    double* h = alloc(nh);
    double* obs = alloc(NS * nobs);
    double* res = alloc(NS * nobs);
    double* ebar = alloc(ne);
    double* hbar = alloc(nh);
    double* lam = alloc(ne);
    double* u = alloc(nh);
    double* w = alloc(std::max(ne, nh));
    kmx_status st = KMX_OK;
    for (double* b : bufs)
        if (!b) st = fail(KMX_E_OOM, "device allocation failed (adjoint working memory)");
    if (bufs.size() != 12) st = fail(KMX_E_OOM, "device allocation failed (adjoint working memory)");
    if (st == KMX_OK) {
        // ---- forward run with checkpoints of (e^n, h^{n-1/2}) every K steps ----
        hipMemsetAsync(e, 0, ne * sizeof(double), s);
        hipMemsetAsync(h, 0, nh * sizeof(double), s);
        for (int n = 0; n < nsteps && st == KMX_OK; ++n) {
            if (n % K == 0) {
                hipMemcpyAsync(ck_e + int64_t(n / K) * ne, e, ne * sizeof(double), hipMemcpyDeviceToDevice, s);
                hipMemcpyAsync(ck_h + int64_t(n / K) * nh, h, nh * sizeof(double), hipMemcpyDeviceToDevice, s);
            }
            st = kmx_step(sp, e, h, J, n * dt, dt, 1, 1, 0, nullptr, stream);
            launch_csr(pr->d_rowptr, pr->d_col, pr->d_val, e, obs + n * nobs, nullptr, int(nobs), 1.0, 0.0, s);
        }
    }
    if (st == KMX_OK) {
        // ---- misfit ----
        const int nb = int(std::min<int64_t>(1024, (NS * nobs + 255) / 256));
        launch_residual(obs, data, res, NS * nobs, sp->d_red, nb, s);
        launch_sum_final(sp->d_red, nb, 1, sp->d_scal, s);
        // ---- reverse sweep ----
        hipMemsetAsync(grad, 0, int64_t(sp->N) * sp->N * sp->N * sizeof(double), s);
        hipMemsetAsync(ebar, 0, ne * sizeof(double), s);
        hipMemsetAsync(hbar, 0, nh * sizeof(double), s);
        launch_csr(pr->d_trowptr, pr->d_tcol, pr->d_tval, res + (NS - 1) * nobs, ebar, pr->d_tidx, pr->ntrows, 1.0,
                   1.0, s);
        PairGradArgs g{};
        space_dims(sp, SP_D, g.lam_dims, g.lam_comp_off);
        space_dims(sp, SP_H, g.h_dims, g.h_comp_off);
        g.metric = sp->d_metric;
        g.metric_mode = sp->metric_mode;
        g.amp = sp->map.kind == 1 ? sp->map.amplitude : 0.0;
        g.axis_tab = sp->d_axis_tab;
        g.inv_eps = sp->d_inv_eps;
        g.tab = sp->d_tab;
        for (int k = 0; k < 4; ++k) g.tab_off[k] = sp->tab_off[k];
        g.ntile = sp->ntile;
        g.npad = sp->npad;
        g.n0 = sp->n0;
        g.n1 = sp->n1;
        g.N = sp->N;
        g.coef = -dt;
        g.grad = grad;
        g.lam = lam;
        for (int seg = nseg - 1; seg >= 0 && st == KMX_OK; --seg) {
            const int n0 = seg * K, n1 = std::min(nsteps, n0 + K);
            hipMemcpyAsync(e, ck_e + int64_t(seg) * ne, ne * sizeof(double), hipMemcpyDeviceToDevice, s);
            hipMemcpyAsync(h, ck_h + int64_t(seg) * nh, nh * sizeof(double), hipMemcpyDeviceToDevice, s);
            for (int n = n0; n < n1 && st == KMX_OK; ++n) {  // recompute the segment, keeping h^{n+1/2}
                st = kmx_step(sp, e, h, J, n * dt, dt, 1, 1, 0, nullptr, stream);
                hipMemcpyAsync(seg_h + int64_t(n - n0) * nh, h, nh * sizeof(double), hipMemcpyDeviceToDevice, s);
            }
            if (st != KMX_OK) break;
            for (int n = n1 - 1; n >= n0; --n) {
                const double t = (n + 0.5) * dt;
                // lam = K1^{-T} ebar
                run_solve(sp, 1, 1, 0, SP_D, ebar, ne, lam, ne, 1.0, 0, 1, nullptr, 0.0, 1, s);
                // hbar += dt D~^{1T} M~ lam
                run_mass(sp, SP_D, false, lam, ne, 1, s);
                run_solve(sp, 1, 0, 1, SP_D, nullptr, 0, w, ne, 1.0, 0, 1, nullptr, 0.0, 0, s);
                run_curlT(sp, 0, w, hbar, dt, s);
                // gradient: -dt / eps_e^2 sum_e Lam . G V   and the dipole terms
                g.h = seg_h + int64_t(n - n0) * nh;
                launch_pair_grad(sp->p, g, s);
                if (J)
                    launch_source_grad(J->d_entries, J->d_prof, J->d_elem, J->n, J->entries_per, lam, J->d_comp_off,
                                       J->d_dims, J->d_inv_eps, t, dt, grad, s);
                // ebar -= dt D^{1T} M K~1^{-T} hbar
                run_solve(sp, 0, 1, 0, SP_B, hbar, nh, u, nh, 1.0, 0, 1, nullptr, 0.0, 1, s);
                run_mass(sp, SP_B, false, u, nh, 1, s);
                run_solve(sp, 0, 0, 1, SP_B, nullptr, 0, w, nh, 1.0, 0, 1, nullptr, 0.0, 0, s);
                run_curlT(sp, 1, w, ebar, -dt, s);
                if (n >= 1)
                    launch_csr(pr->d_trowptr, pr->d_tcol, pr->d_tval, res + int64_t(n - 1) * nobs, ebar, pr->d_tidx,
                               pr->ntrows, 1.0, 1.0, s);
            }
        }
        double sumsq = 0.0;
        hipMemcpyAsync(&sumsq, sp->d_scal, sizeof(double), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess && st == KMX_OK) st = fail(KMX_E_DEVICE, "adjoint run failed");
        if (st == KMX_OK) *loss_host = 0.5 * sumsq;
        if (st == KMX_OK && hipGetLastError() != hipSuccess) st = fail(KMX_E_DEVICE, "kernel launch failed");
    }
    hipStreamSynchronize(s);
    for (double* b : bufs) hipFree(b);
    return st;
}

kmx_status kmx_init_stagger(kmx_space* sp, const double* E, double* H, double dt, int batch, int flags,
                            void* stream) {
    if (!sp || !E || !H) return fail(KMX_E_ARG, "NULL argument");
    if (batch < 1 || batch > sp->max_batch) return fail(KMX_E_ARG, "batch out of range");
    const int track = flags & KMX_TRACK_DB;
    const int64_t es = sp->n_e * (1 + track), hs = sp->n_h * (1 + track);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (track && sp->lift_n) return fail(KMX_E_ARG, "tracking d and b with a lifting is not supported");
    if (track) run_curl(sp, 1, E, es, H + sp->n_h, hs, 0.5 * dt, 1.0, batch, s);
    run_mass(sp, SP_B, true, E, es, batch, s);
    run_solve(sp, 0, 0, 1, SP_B, nullptr, 0, H, hs, 0.5 * dt, 1, batch, nullptr, 0.0, 1, s);
    // the lifting at t = 0: h += dt/2 sum_j g_j(0) v_h^j
    if (sp->lift_n)
        launch_lift(H, hs, sp->d_lift_vh, sp->n_h, lift_terms(sp), 0.0, 0.0, nullptr, -0.5 * dt, 0, batch, s);
    CHECK_LAUNCH();
    return KMX_OK;
}

// The leapfrog loop.  With t_dev the source time of step n is *t_dev +
// (n + 1/2) dt (graph replay), otherwise t_start + (n + 1/2) dt.
// x = K^{-1} y (or K^{-T} y) in mixed precision: three FP32 mode products with
// the dense inverse factors, then `refine_steps` corrections with the FP64
// banded residual; out = (accumulate ? out : 0) + alpha * x.  y: FP64 field of
// the K layout with stride nfield (left unchanged); out may not alias y.
void mixed_solve(kmx_space* sp, int which_K1, int transpose, const double* y, double* out, int64_t out_stride,
                 double alpha, int accumulate, int batch, hipStream_t s) {
    const int64_t nf = std::max(sp->n_e, sp->n_h);
    const int layout = which_K1 ? SP_D : SP_B;
    ModeArgs m{};
    space_dims(sp, layout, m.dims, m.comp_off);
    m.in_stride = m.out_stride = nf;
    m.A = sp->d_inv32;
    m.alpha = 1.0;
    auto apply3 = [&](const double* in, double* dst, int kind) {
        ProfScope ps(sp, s, PK_MODE);
        for (int ax = 0; ax < 3; ++ax) {
            for (int c = 0; c < 3; ++c) m.A_off[c] = sp->inv32_off[pair_fac(which_K1, transpose, c, ax)];
            m.axis = ax;
            m.in = ax == 0 ? static_cast<const void*>(in) : (ax == 1 ? sp->d_m32a : sp->d_m32b);
            m.in_f64 = ax == 0;
            m.out = ax == 0 ? static_cast<void*>(sp->d_m32a) : (ax == 1 ? static_cast<void*>(sp->d_m32b) : dst);
            m.out_kind = ax < 2 ? 0 : kind;
            launch_mode(m, batch, s);
        }
    };
    apply3(y, sp->d_mx, 1);
    for (int it = 0; it < sp->refine_steps; ++it) {
        (void)hipMemcpy2DAsync(sp->d_mr, nf * sizeof(double), y, nf * sizeof(double),
                               size_t(which_K1 ? sp->n_e : sp->n_h) * sizeof(double), batch,
                               hipMemcpyDeviceToDevice, s);
        run_solve(sp, which_K1, transpose, 0, layout, sp->d_mx, nf, sp->d_mr, nf, -1.0, 1, batch, nullptr, 0.0, 2, s);
        apply3(sp->d_mr, sp->d_mx, 2);
    }
    const int64_t n = which_K1 ? sp->n_e : sp->n_h;
    if (accumulate) {
        launch_strided_axpy(sp->d_mx, nf, out, out_stride, n, alpha, batch, s);
    } else {
        for (int b = 0; b < batch; ++b)
            (void)hipMemcpyAsync(out + b * out_stride, sp->d_mx + b * nf, n * sizeof(double), hipMemcpyDeviceToDevice,
                                 s);
        if (alpha != 1.0) launch_strided_axpy(sp->d_mx, nf, out, out_stride, n, alpha - 1.0, batch, s);
    }
}

// out += alpha * K^{-1} y by three FP64 mode products with the dense inverse
// factors on the matrix cores.  y: d_tmp2 layout (stride nfield); d_tmp2 and
// d_tmp are overwritten.
void dense_solve(kmx_space* sp, int which_K1, const double* y, double* out, int64_t out_stride, double alpha,
                 int batch, const kmx_source* J, double t_src, const double* t_dev, hipStream_t s) {
    const int64_t nf = std::max(sp->n_e, sp->n_h);
    DenseArgs a{};
    space_dims(sp, which_K1 ? SP_D : SP_B, a.dims, a.comp_off);
    a.frag = sp->d_frag64;
    for (int c = 0; c < 3; ++c)
        for (int ax = 0; ax < 3; ++ax) a.frag_off[c][ax] = sp->frag64_off[pair_fac(which_K1, 0, c, ax)];
    if (J) {
        a.src_entries = J->d_entries;
        a.src_prof = J->d_prof;
        a.src_off = reinterpret_cast<const int*>(J->d_prof + 4 * J->n);
        a.n_src = J->n;
        a.entries_per = J->entries_per;
        a.t_src = t_src;
        a.t_dev = t_dev;
    }
    ProfScope ps(sp, s, PK_DENSE);
    a.in = y;
    a.in_stride = nf;
    a.out = sp->d_tmp;
    a.out_stride = nf;
    launch_dense_xy(a, batch, s);
    a.in = sp->d_tmp;
    a.out = out;
    a.out_stride = out_stride;
    a.alpha = alpha;
    a.accumulate = 1;
    a.n_src = 0;
    launch_dense_z(a, batch, s);
}

// Whether the separable persistent kernel can run a step call: identity map,
// eps and mu the same in every element, no per-step energy output, lines that
// fit the kernel's registers and component tensors that fit one workgroup's LDS.
bool sep_eligible(const kmx_space* sp, const double* energy_dev) {
    if (sp->map.kind != 0 || !sp->uniform_eps || !sp->uniform_mu || energy_dev || sp->lift_n) return false;
    if (sp->precision == KMX_MIXED) return false;
    if (sep_line_max(std::max(sp->n0, sp->n1)) == 0) return false;
    int ed[3][3], hd[3][3];
    int64_t o[3];
    space_dims(sp, SP_E, ed, o);
    space_dims(sp, SP_H, hd, o);
    return sep_lds_bytes(ed, hd) <= size_t(sp->max_lds);
}

// Batches from this size up take the separable kernel when no plan is set
// (one workgroup per member; small batches leave most compute units idle).
constexpr int SEP_AUTO_MIN_BATCH = 32;

kmx_status run_sep(kmx_space* sp, double* E, double* H, const kmx_source* J, double t_start, const double* t_dev,
                   double dt, int nsteps, int batch, int track, hipStream_t s) {
    SepArgs a{};
    a.n_e = sp->n_e;
    a.n_h = sp->n_h;
    a.track = track;
    a.e_stride = sp->n_e * (1 + track);
    a.h_stride = sp->n_h * (1 + track);
    space_dims(sp, SP_E, a.edims, a.e_off);
    space_dims(sp, SP_H, a.hdims, a.h_off);
    for (int k = 0; k < 4; ++k) {
        a.gram_off[k] = sp->gram_off[k];
        a.fac_off[k] = sp->fac_off[k];
    }
    a.inv_mu = sp->mu_value;
    a.inv_eps = sp->eps_value;
    a.dt = dt;
    a.nsteps = nsteps;
    a.t_start = t_start;
    a.t_dev = t_dev;
    if (J) {
        a.src_entries = J->d_entries;
        a.src_prof = J->d_prof;
        a.src_off = reinterpret_cast<const int*>(J->d_prof + 4 * J->n);
        a.n_src = J->n;
        a.entries_per = J->entries_per;
    }
    ProfScope ps(sp, s, PK_SEP);
    const hipError_t err = launch_sep(sp->p, sep_line_max(std::max(sp->n0, sp->n1)),
                                      sp->plan_kind == KMX_PLAN_SEPARABLE_FUSED ? 1 : 0, E, H, sp->d_gram, sp->d_fac,
                                      a, batch, sp->plan_threads, s);
    if (err != hipSuccess) return fail(KMX_E_DEVICE, std::string("separable kernel: ") + hipGetErrorString(err));
    return KMX_OK;
}

// One kick-drift substep of the tiled plans:
//   h -= ka K~1^{-1} M D^1 e   (b -= ka D^1 e when tracking)
//   e += kb K1^{-1} (M~ D~^1 h - s(t_half))   (d += kb D~^1 h)
// the leapfrog step with ka = kb = dt, a substep of a composition otherwise.
// t_base + t_step (or *t_dev + t_step under graph replay) is the time at the
// start of the substep, the lifting's t_n; t_half the source time.
// keep_w: also update the kept images K~1 h (d_wh) and K1 e (d_we) of the
// per-step energy with the gathered mass applies.
static void tiled_substep(kmx_space* sp, double* E, double* H, int64_t es, int64_t hs, double ka, double kb, int batch,
                   int track, bool dense, bool mixed, const kmx_source* J, double t_half, const double* t_dev,
                   hipStream_t s, double t_base = 0.0, double t_step = 0.0, bool keep_w = false) {
    const int64_t nf = std::max(sp->n_e, sp->n_h);
    double* wh = keep_w ? sp->d_wh : nullptr;
    double* we = keep_w ? sp->d_we : nullptr;
    // M D^1 e (and b -= ka D^1 e), then h -= ka K~1^{-1} (.)
    run_mass(sp, SP_B, true, E, es, batch, s, track ? H + sp->n_h : nullptr, hs, -ka);
    if (dense && !mixed) {
        run_solve(sp, 0, 0, 1, SP_B, nullptr, 0, sp->d_tmp2, nf, 1.0, 0, batch, nullptr, 0.0, 0, s, nullptr, nullptr,
                  wh, sp->n_h, -ka);
        dense_solve(sp, 0, sp->d_tmp2, H, hs, -ka, batch, nullptr, 0.0, nullptr, s);
    } else if (mixed) {
        run_solve(sp, 0, 0, 1, SP_B, nullptr, 0, sp->d_my, nf, 1.0, 0, batch, nullptr, 0.0, 0, s, nullptr, nullptr, wh,
                  sp->n_h, -ka);
        mixed_solve(sp, 0, 0, sp->d_my, H, hs, -ka, 1, batch, s);
    } else {
        run_solve(sp, 0, 0, 1, SP_B, nullptr, 0, H, hs, -ka, 1, batch, nullptr, 0.0, 1, s, nullptr, nullptr, wh, sp->n_h,
                  -ka);
    }
    // the lifting: h -= ka sum_j g_j(t_n) v_h^j (t_n = t_half - ka / 2)
    if (sp->lift_n)
        launch_lift(H, hs, sp->d_lift_vh, sp->n_h, lift_terms(sp), t_base, t_step, t_dev, ka, 0, batch, s);
    // M~ D~^1 h (and d += kb D~^1 h), then e += kb K1^{-1} (. - s); a pattern
    // source is subtracted from the gathered field, point dipoles inside the
    // solve's first pass
    run_mass(sp, SP_D, true, H, hs, batch, s, track ? E + sp->n_e : nullptr, es, kb);
    const bool pattern = J && J->kind == 1;
    const kmx_source* Jd = pattern ? nullptr : J;
    auto sub_pattern = [&](double* y) {
        launch_pattern_source(y, nf, J->d_pattern, J->npat > 1 ? sp->n_e : 0, sp->n_e, J->d_series, J->nsamples,
                              J->ts0, J->tsh, t_dev, t_half, batch, s);
    };
    if (dense && !mixed) {
        run_solve(sp, 1, 0, 1, SP_D, nullptr, 0, sp->d_tmp2, nf, 1.0, 0, batch, nullptr, 0.0, 0, s, nullptr, nullptr,
                  we, sp->n_e, kb);
        if (pattern) sub_pattern(sp->d_tmp2);
        dense_solve(sp, 1, sp->d_tmp2, E, es, kb, batch, Jd, t_half, t_dev, s);
    } else if (mixed) {
        run_solve(sp, 1, 0, 1, SP_D, nullptr, 0, sp->d_my, nf, 1.0, 0, batch, Jd, t_half, 0, s, nullptr, t_dev, we,
                  sp->n_e, kb);
        if (pattern) sub_pattern(sp->d_my);
        mixed_solve(sp, 1, 0, sp->d_my, E, es, kb, 1, batch, s);
    } else if (pattern) {
        run_solve(sp, 1, 0, 1, SP_D, nullptr, 0, sp->d_tmp2, nf, 1.0, 0, batch, nullptr, 0.0, 0, s);
        sub_pattern(sp->d_tmp2);
        run_solve(sp, 1, 0, 0, SP_D, sp->d_tmp2, nf, E, es, kb, 1, batch, nullptr, 0.0, 1, s);
    } else {
        run_solve(sp, 1, 0, 1, SP_D, nullptr, 0, E, es, kb, 1, batch, J, t_half, 1, s, nullptr, t_dev, we, sp->n_e, kb);
    }
    // the lifting: e -= sum_j (g_j(t_n + kb) - g_j(t_n)) v_e^j
    if (sp->lift_n)
        launch_lift(E, es, sp->d_lift_ve, sp->n_e, lift_terms(sp), t_base, t_step, t_dev, kb, 1, batch, s);
}

kmx_status step_loop(kmx_space* sp, double* E, double* H, const kmx_source* J, double t_start, const double* t_dev,
                     double dt, int nsteps, int batch, int flags, double* energy_dev, hipStream_t s) {
    if (!sp || !E || !H) return fail(KMX_E_ARG, "NULL argument");
    if (batch < 1 || batch > sp->max_batch) return fail(KMX_E_ARG, "batch out of range");
    if (nsteps < 0) return fail(KMX_E_ARG, "nsteps < 0");
    if (!std::isfinite(dt)) return fail(KMX_E_ARG, "dt not finite");
    if (sp->dt_cfl > 0.0 && std::fabs(dt) > sp->dt_cfl) return fail(KMX_E_UNSTABLE, "|dt| above the CFL limit");
    const int track = flags & KMX_TRACK_DB;
    if (J && J->sp != sp) return fail(KMX_E_ARG, "source belongs to another space");
    if (J && track) return fail(KMX_E_ARG, "tracking d and b needs J = NULL (d would need M~^{-1} s)");
    if (sp->lift_n && track) return fail(KMX_E_ARG, "tracking d and b with a lifting is not supported");
    if (energy_dev && !track) return fail(KMX_E_ARG, "energy output needs KMX_TRACK_DB");
    if (J && J->kind == 1 && J->npat > 1 && batch > J->npat)
        return fail(KMX_E_ARG, "the source has fewer patterns than the batch has members");
    // (the separable plan takes point dipoles only)
    const bool sep_ok = sep_eligible(sp, energy_dev) && !(J && J->kind == 1);
    int kind = sp->plan_kind;
    if ((kind == KMX_PLAN_SEPARABLE || kind == KMX_PLAN_SEPARABLE_FUSED) && !sep_ok)
        return fail(KMX_E_STATE, "separable plan needs the identity map, uniform eps and mu, no energy output, "
                                 "point-dipole sources only and component tensors that fit one workgroup's LDS");
    if (kind == KMX_PLAN_AUTO) kind = (sep_ok && batch >= SEP_AUTO_MIN_BATCH) ? KMX_PLAN_SEPARABLE : KMX_PLAN_TILED;
    if (kind == KMX_PLAN_SEPARABLE || kind == KMX_PLAN_SEPARABLE_FUSED) {
        if (nsteps > 0) {
            const kmx_status st = run_sep(sp, E, H, J, t_start, t_dev, dt, nsteps, batch, track, s);
            if (st != KMX_OK) return st;
        }
        if (t_dev) launch_advance_time(const_cast<double*>(t_dev), nsteps * dt, s);
        CHECK_LAUNCH();
        return KMX_OK;
    }
    const int64_t es = sp->n_e * (1 + track), hs = sp->n_h * (1 + track);
    const bool mixed = sp->precision == KMX_MIXED;
    const bool dense = kind == KMX_PLAN_TILED_DENSE;
    sp->mass_waves4 = kind == KMX_PLAN_TILED_W4 ? 1 : 0;
    // per-step energy: the images K1 e and K~1 h of the call's first state,
    // then kept up to date by the substeps with the mass applies they gather
    if (energy_dev && nsteps > 0) {
        run_solve(sp, 1, 0, 0, SP_D, E, es, sp->d_we, sp->n_e, 1.0, 0, batch, nullptr, 0.0, 2, s);
        run_solve(sp, 0, 0, 0, SP_B, H, hs, sp->d_wh, sp->n_h, 1.0, 0, batch, nullptr, 0.0, 2, s);
    }
    for (int n = 0; n < nsteps; ++n) {
        const double t_half = (t_dev ? 0.0 : t_start) + (n + 0.5) * dt;
        tiled_substep(sp, E, H, es, hs, dt, dt, batch, track, dense, mixed, J, t_half, t_dev, s, t_dev ? 0.0 : t_start,
                      n * dt, energy_dev != nullptr);
        if (energy_dev) run_energy_dots(sp, E, H, dt, batch, n, energy_dev + int64_t(n) * batch, s);
    }
    if (energy_dev && nsteps > 0)
        finish_energy_dots(sp, dt, batch, nsteps - 1, energy_dev + int64_t(nsteps - 1) * batch, s);
    if (t_dev) launch_advance_time(const_cast<double*>(t_dev), nsteps * dt, s);
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_step(kmx_space* sp, double* E, double* H, const kmx_source* J, double t_start, double dt,
                    int nsteps, int batch, int flags, double* energy_dev, void* stream) {
    return step_loop(sp, E, H, J, t_start, nullptr, dt, nsteps, batch, flags, energy_dev,
                     static_cast<hipStream_t>(stream));
}

// Weights c_1..c_m of the symmetric triple-jump composition of the leapfrog
// of the given even order (2: the leapfrog; 2k+2: z1, z0, z1 times the order-2k
// weights, z1 = 1 / (2 - 2^(1/(2k+1))), z0 = 1 - 2 z1).
static std::vector<double> composition_weights(int order) {
    std::vector<double> c{1.0};
    for (int k = 1; k < order / 2; ++k) {
        const double z1 = 1.0 / (2.0 - std::pow(2.0, 1.0 / (2 * k + 1))), z0 = 1.0 - 2.0 * z1;
        std::vector<double> n;
        for (double z : {z1, z0, z1})
            for (double w : c) n.push_back(w * z);
        c.swap(n);
    }
    return c;
}

kmx_status kmx_init_split(kmx_space* sp, const double* E, double* H, double dt, int order, int batch, int flags,
                          void* stream) {
    if (order != 2 && order != 4 && order != 6) return fail(KMX_E_ARG, "order must be 2, 4 or 6");
    return kmx_init_stagger(sp, E, H, composition_weights(order)[0] * dt, batch, flags, stream);
}

kmx_status kmx_step_split(kmx_space* sp, double* E, double* H, double dt, int nsteps, int order, int batch,
                          int flags, void* stream) {
    if (!sp || !E || !H) return fail(KMX_E_ARG, "NULL argument");
    if (order != 2 && order != 4 && order != 6) return fail(KMX_E_ARG, "order must be 2, 4 or 6");
    if (batch < 1 || batch > sp->max_batch) return fail(KMX_E_ARG, "batch out of range");
    if (nsteps < 0) return fail(KMX_E_ARG, "nsteps < 0");
    if (!std::isfinite(dt)) return fail(KMX_E_ARG, "dt not finite");
    if (sp->lift_n) return fail(KMX_E_STATE, "composed steps do not take a lifting");
    const std::vector<double> c = composition_weights(order);
    double cmax = 0.0;
    for (double w : c) cmax = std::max(cmax, std::fabs(w));
    if (sp->dt_cfl > 0.0 && cmax * std::fabs(dt) > sp->dt_cfl)
        return fail(KMX_E_UNSTABLE, "the largest substep |c_j dt| is above the CFL limit");
    int kind = sp->plan_kind;
    if (kind == KMX_PLAN_SEPARABLE || kind == KMX_PLAN_SEPARABLE_FUSED)
        return fail(KMX_E_STATE, "composed steps run the tiled plans only");
    if (kind == KMX_PLAN_AUTO) kind = KMX_PLAN_TILED;
    const int track = flags & KMX_TRACK_DB;
    const int64_t es = sp->n_e * (1 + track), hs = sp->n_h * (1 + track);
    const bool mixed = sp->precision == KMX_MIXED;
    const bool dense = kind == KMX_PLAN_TILED_DENSE;
    sp->mass_waves4 = kind == KMX_PLAN_TILED_W4 ? 1 : 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int n = 0; n < nsteps; ++n)
        for (size_t j = 0; j < c.size(); ++j) {
            // the first kick also carries the previous step's last half kick (c_m = c_1)
            const double a = j == 0 ? c[0] : 0.5 * (c[j - 1] + c[j]);
            tiled_substep(sp, E, H, es, hs, a * dt, c[j] * dt, batch, track, dense, mixed, nullptr, 0.0, nullptr, s);
        }
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_set_time(kmx_space* sp, double t, void* stream) {
    if (!sp) return fail(KMX_E_ARG, "space is NULL");
    HIP_TRY(hipMemcpyAsync(sp->d_time, &t, sizeof(double), hipMemcpyHostToDevice, static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return KMX_OK;
}

kmx_status kmx_get_time(kmx_space* sp, double* t, void* stream) {
    if (!sp || !t) return fail(KMX_E_ARG, "NULL argument");
    HIP_TRY(hipMemcpyAsync(t, sp->d_time, sizeof(double), hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return KMX_OK;
}

kmx_status kmx_set_refinement(kmx_space* sp, int steps) {
    if (!sp || steps < 0 || steps > 8) return fail(KMX_E_ARG, "refinement steps must be 0..8");
    sp->refine_steps = steps;
    return KMX_OK;
}

kmx_status kmx_set_plan(kmx_space* sp, int kind, int threads) {
    if (!sp) return fail(KMX_E_ARG, "space is NULL");
    if (kind != KMX_PLAN_AUTO && kind != KMX_PLAN_TILED && kind != KMX_PLAN_SEPARABLE &&
        kind != KMX_PLAN_SEPARABLE_FUSED && kind != KMX_PLAN_TILED_DENSE && kind != KMX_PLAN_TILED_W4)
        return fail(KMX_E_ARG, "unknown plan kind");
    if (threads < 64 || threads > SEP_MAX_THREADS || threads % 64)
        return fail(KMX_E_ARG, "threads must be 64..768, a multiple of 64");
    if (kind == KMX_PLAN_TILED_DENSE && !sp->dense_ok)
        return fail(KMX_E_ARG, "the tiled-dense plan needs lines of at most 80 entries and its LDS on the device");
    sp->plan_kind = kind;
    sp->plan_threads = threads;
    return KMX_OK;
}

kmx_status kmx_get_plan(const kmx_space* sp, int* kind, int* threads) {
    if (!sp || !kind || !threads) return fail(KMX_E_ARG, "NULL argument");
    *kind = sp->plan_kind;
    *threads = sp->plan_threads;
    return KMX_OK;
}

kmx_status kmx_tune(kmx_space* sp, int batch, int probe_steps, const kmx_source* J, double dt, double* ms_out,
                    void* stream) {
    if (!sp || batch < 1 || batch > sp->max_batch || probe_steps < 1) return fail(KMX_E_ARG, "bad argument");
    if (sp->prof_on) return fail(KMX_E_STATE, "profiling is on");
    hipStream_t s = static_cast<hipStream_t>(stream);
    static const int cand_kind[KMX_TUNE_CANDIDATES] = {
        KMX_PLAN_TILED,     KMX_PLAN_TILED_W4,  KMX_PLAN_TILED_DENSE,     KMX_PLAN_SEPARABLE,
        KMX_PLAN_SEPARABLE, KMX_PLAN_SEPARABLE, KMX_PLAN_SEPARABLE_FUSED, KMX_PLAN_SEPARABLE_FUSED};
    static const int cand_threads[KMX_TUNE_CANDIDATES] = {0, 0, 0, 384, 512, 768, 512, 768};
    const bool sep_ok = sep_eligible(sp, nullptr);
    double* E = nullptr;
    double* H = nullptr;
    if (hipMalloc(&E, size_t(batch) * sp->n_e * sizeof(double)) != hipSuccess ||
        hipMalloc(&H, size_t(batch) * sp->n_h * sizeof(double)) != hipSuccess) {
        if (E) (void)hipFree(E);
        return fail(KMX_E_OOM, "device allocation failed (tuning fields)");
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    const int saved_kind = sp->plan_kind, saved_threads = sp->plan_threads;
    kmx_status st = KMX_OK;
    double best = 1e300;
    int best_k = 0;
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) st = fail(KMX_E_DEVICE, "events");
    (void)hipMemsetAsync(E, 0, size_t(batch) * sp->n_e * sizeof(double), s);
    (void)hipMemsetAsync(H, 0, size_t(batch) * sp->n_h * sizeof(double), s);
    for (int k = 0; k < KMX_TUNE_CANDIDATES && st == KMX_OK; ++k) {
        double ms = -1.0;
        if ((k < 3 && (cand_kind[k] != KMX_PLAN_TILED_DENSE || sp->dense_ok)) || (k >= 3 && sep_ok)) {
            sp->plan_kind = cand_kind[k];
            sp->plan_threads = k < 3 ? saved_threads : cand_threads[k];
            st = step_loop(sp, E, H, J, 0.0, nullptr, dt, 1, batch, 0, nullptr, s);  // warm-up
            if (st == KMX_OK) (void)hipEventRecord(ev[0], s);
            if (st == KMX_OK) st = step_loop(sp, E, H, J, 0.0, nullptr, dt, probe_steps, batch, 0, nullptr, s);
            if (st == KMX_OK) (void)hipEventRecord(ev[1], s);
            float f = 0.0f;
            if (st == KMX_OK && (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&f, ev[0], ev[1]) != hipSuccess))
                st = fail(KMX_E_DEVICE, "tuning run failed");
            if (st == KMX_OK) {
                ms = double(f) / probe_steps;
                if (ms < best) {
                    best = ms;
                    best_k = k;
                }
            }
        }
        if (ms_out) ms_out[k] = ms;
    }
    (void)hipStreamSynchronize(s);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(E);
    (void)hipFree(H);
    if (st != KMX_OK) {
        sp->plan_kind = saved_kind;
        sp->plan_threads = saved_threads;
        return st;
    }
    sp->plan_kind = cand_kind[best_k];
    sp->plan_threads = best_k < 3 ? saved_threads : cand_threads[best_k];
    return KMX_OK;
}

kmx_status kmx_graph_create(kmx_space* sp, double* E, double* H, const kmx_source* J, double dt, int nsteps,
                            int batch, int flags, double* energy_dev, kmx_graph** out) {
    if (!sp || !out || nsteps < 1) return fail(KMX_E_ARG, "bad argument");
    if (sp->prof_on) return fail(KMX_E_STATE, "profiling is on; graphs are captured without timing events");
    *out = nullptr;
    if (!sp->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&sp->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = sp->capture_stream;
    HIP_TRY(hipStreamSynchronize(cs));
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    kmx_status st = step_loop(sp, E, H, J, 0.0, sp->d_time, dt, nsteps, batch, flags, energy_dev, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (st != KMX_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (ec != hipSuccess) return fail(KMX_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        hipGraphDestroy(graph);
        return fail(KMX_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    kmx_graph* g = new kmx_graph();
    ++sp->live_graphs;
    g->sp = sp;
    g->graph = graph;
    g->exec = exec;
    g->nsteps = nsteps;
    *out = g;
    return KMX_OK;
}

kmx_status kmx_graph_launch(kmx_graph* g, void* stream) {
    if (!g) return fail(KMX_E_ARG, "graph is NULL");
    HIP_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return KMX_OK;
}

void kmx_graph_destroy(kmx_graph* g) {
    if (!g) return;
    {
        std::lock_guard<std::mutex> lk(g_spaces_mu);
        if (g->sp && g_spaces.count(g->sp)) --g->sp->live_graphs;
    }
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

kmx_status kmx_energy(kmx_space* sp, const double* E, const double* H, double dt, int batch, double* out_host,
                      void* stream) {
    if (!sp || !E || !H || !out_host) return fail(KMX_E_ARG, "NULL argument");
    if (batch < 1 || batch > sp->max_batch) return fail(KMX_E_ARG, "batch out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    run_energy(sp, E, H, dt, batch, sp->d_scal, 2, s);
    CHECK_LAUNCH();
    std::vector<double> tmp(2 * batch);
    HIP_TRY(hipMemcpyAsync(tmp.data(), sp->d_scal, 2 * batch * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < 2 * batch; ++k) out_host[k] = tmp[k];
    for (int k = 0; k < batch; ++k)
        if (!std::isfinite(tmp[2 * k])) return fail(KMX_E_UNSTABLE, "energy is not finite");
    return KMX_OK;
}

kmx_status kmx_op_curl(kmx_space* sp, int which, const double* x, double* y, void* stream) {
    if (!sp || !x || !y || (which != 0 && which != 1)) return fail(KMX_E_ARG, "bad argument");
    run_curl(sp, which == 0, x, 0, y, 0, 1.0, 0.0, 1, static_cast<hipStream_t>(stream));
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_op_mass(kmx_space* sp, int which, int curl, const double* x, double* y, void* stream) {
    if (!sp || !x || !y || (which != 0 && which != 1)) return fail(KMX_E_ARG, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int space = which == 0 ? SP_B : SP_D;
    run_mass(sp, space, curl != 0, x, 0, 1, s);
    run_solve(sp, which, 0, 1, space, nullptr, 0, y, 0, 1.0, 0, 1, nullptr, 0.0, 0, s);
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_op_solve(kmx_space* sp, int which, int transpose, const double* y, double* x, void* stream) {
    if (!sp || !x || !y || (which != 0 && which != 1)) return fail(KMX_E_ARG, "bad argument");
    if (sp->precision == KMX_MIXED)
        mixed_solve(sp, which, transpose != 0, y, x, 0, 1.0, 0, 1, static_cast<hipStream_t>(stream));
    else
        run_solve(sp, which, transpose != 0, 0, which ? SP_D : SP_B, y, 0, x, 0, 1.0, 0, 1, nullptr, 0.0, 1,
                  static_cast<hipStream_t>(stream));
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_op_pairing(kmx_space* sp, int which, const double* x, double* y, void* stream) {
    if (!sp || !x || !y || (which != 0 && which != 1)) return fail(KMX_E_ARG, "bad argument");
    run_solve(sp, which, 0, 0, which ? SP_D : SP_B, x, 0, y, 0, 1.0, 0, 1, nullptr, 0.0, 2,
              static_cast<hipStream_t>(stream));
    CHECK_LAUNCH();
    return KMX_OK;
}

}  // extern "C"

// ===========================================================================
// The first scheme (Section 3.3): Hodge stars with the 1-form mass matrices,
//   M^1_eps d_t e = K1^T D~^1 h,   M~^1_mu d_t h = - K~1^T D^1 e,
// each mass system solved by preconditioned conjugate gradients.  The
// preconditioner is a Kronecker-product approximation of the mass matrix (1D
// Gram matrices weighted by a separable fit of the metric and the material,
// s1_build_precond): its inverse is applied with dense inverse factors on the
// matrix cores, as are the transposed pairing matrices (the same dense plane
// and z passes as the tiled-dense plan's solves).
// ===========================================================================
namespace {

// work vectors of the first scheme, each max(n_e, n_h) long
enum { S1_Y = 0, S1_R, S1_Z, S1_P, S1_AP, S1_CU, S1_XE, S1_XH, S1_VECS };

double* s1_vec(kmx_space* sp, int k) { return sp->d_s1 + int64_t(k) * std::max(sp->n_e, sp->n_h); }

kmx_status s1_upload_padded(kmx_space* sp, double** dst, const std::vector<double>& v) {
    const int N = sp->N, P = sp->npad;
    std::vector<double> pad(size_t(P) * P * P, 0.0);
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x)
                pad[(size_t(z) * P + y) * P + x] = v.empty() ? 1.0 : v[(size_t(z) * N + y) * N + x];
    if (!*dst && hipMalloc(dst, pad.size() * sizeof(double)) != hipSuccess)
        return fail(KMX_E_OOM, "device allocation failed (first-scheme materials)");
    HIP_TRY(hipMemcpy(*dst, pad.data(), pad.size() * sizeof(double), hipMemcpyHostToDevice));
    return KMX_OK;
}

// 1D Gram matrix of one tag with a weight per global Gauss point of the axis
std::vector<double> gram_weighted(const Tables& tb, int tag, const std::vector<double>& f) {
    const int n = (tag == PV || tag == DD) ? tb.n0 : tb.n1;
    const int K = tag_support(tb.p, tag);
    std::vector<double> G(size_t(n) * n, 0.0);
    for (int e = 0; e < tb.N; ++e)
        for (int q = 0; q < tb.nq; ++q) {
            const double* v = &tb.tab[tag][(e * tb.nq + q) * K];
            const double w = tb.wq[e * tb.nq + q] * f[e * tb.nq + q];
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) {
                    const int gi = e + i + tag_offset(tag), gj = e + j + tag_offset(tag);
                    if (gi < 0 || gj < 0 || gi >= n || gj >= n) continue;
                    G[size_t(gi) * n + gj] += w * v[i] * v[j];
                }
        }
    return G;
}

// The preconditioner of the 1-form mass solves: for each space (E with eps, H
// with mu) and component c, the diagonal entry gamma_e (G1)_cc of the weighted
// metric is fitted by a separable product fx(x) fy(y) fz(z) (the best additive
// fit of its logarithm: the mean over the other two axes, less two thirds of
// the overall mean); block c of the preconditioner is then the Kronecker
// product of the 1D Gram matrices weighted by fx, fy, fz, inverted exactly.
// For the identity map and uniform materials it is the mass matrix itself.
kmx_status s1_build_precond(kmx_space* sp) {
    const Tables& tb = sp->tb;
    const int N = tb.N, nq = tb.nq, M = N * nq;
    std::vector<double> lm[2][3][3];
    double tot[2][3] = {};
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) lm[s][c][a].assign(M, 0.0);
    for (int ez = 0; ez < N; ++ez)
        for (int ey = 0; ey < N; ++ey)
            for (int ex = 0; ex < N; ++ex) {
                const size_t el = (size_t(ez) * N + ey) * N + ex;
                const double gam[2] = {sp->eps_host.empty() ? 1.0 : sp->eps_host[el],
                                       sp->mu_host.empty() ? 1.0 : sp->mu_host[el]};
                for (int iz = 0; iz < nq; ++iz)
                    for (int iy = 0; iy < nq; ++iy)
                        for (int ix = 0; ix < nq; ++ix) {
                            const int64_t q = ((((int64_t(ez) * N + ey) * N + ex) * nq + iz) * nq + iy) * nq + ix;
                            const double xh[3] = {tb.xq[ex * nq + ix], tb.xq[ey * nq + iy], tb.xq[ez * nq + iz]};
                            double J[9], S[3][3];
                            map_jacobian(sp, q, xh, J);
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j)
                                    S[i][j] = J[i] * J[j] + J[3 + i] * J[3 + j] + J[6 + i] * J[6 + j];
                            const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                                               J[2] * (J[3] * J[7] - J[4] * J[6]);
                            const int g3[3] = {ex * nq + ix, ey * nq + iy, ez * nq + iz};
                            for (int c = 0; c < 3; ++c) {
                                // (det DF (DF^T DF)^{-1})_cc = cofactor_cc(S) / det DF
                                const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
                                const double g1 = (S[c1][c1] * S[c2][c2] - S[c1][c2] * S[c2][c1]) / det;
                                for (int s = 0; s < 2; ++s) {
                                    const double lg = std::log(gam[s] * g1);
                                    tot[s][c] += lg;
                                    for (int a = 0; a < 3; ++a) lm[s][c][a][g3[a]] += lg;
                                }
                            }
                        }
            }
    std::vector<double> frag;
    const double m2 = double(M) * M, m3 = m2 * M;
    for (int s = 0; s < 2; ++s) {
        const int space = s == 0 ? SP_E : SP_H;
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) {
                std::vector<double> f(M);
                for (int i = 0; i < M; ++i) f[i] = std::exp(lm[s][c][a][i] / m2 - (2.0 / 3.0) * tot[s][c] / m3);
                const int tag = space_tag(space, c, a);
                const int n = (tag == PV || tag == DD) ? sp->n0 : sp->n1;
                const std::vector<double> inv = dense_inverse(gram_weighted(tb, tag, f), n);
                sp->frag_pre_off[s][c][a] = int64_t(frag.size());
                frag.resize(frag.size() + size_t(dense_frag_doubles(n)));
                dense_fragments(inv.data(), n, frag.data() + sp->frag_pre_off[s][c][a]);
            }
    }
    // rebuilt into the same allocation (its size depends on p and N only), so
    // device pointers taken earlier stay valid
    if (sp->d_frag_pre && sp->frag_pre_len == int64_t(frag.size())) {
        HIP_TRY(hipMemcpy(sp->d_frag_pre, frag.data(), frag.size() * sizeof(double), hipMemcpyHostToDevice));
        return KMX_OK;
    }
    if (sp->d_frag_pre) return fail(KMX_E_STATE, "preconditioner size changed");
    sp->frag_pre_len = int64_t(frag.size());
    return upload(&sp->d_frag_pre, frag);
}

// Set-up at the first use (and after kmx_set_materials): eps and mu padded to
// the tiles, the 1-form metric factor when the metric is streamed, and the
// work vectors.  Synchronous; not for use under graph capture.
kmx_status s1_prepare(kmx_space* sp) {
    if (!sp->dense_ok) return fail(KMX_E_STATE, "the first scheme needs the dense FP64 kernels (LDS too small)");
    kmx_status st;
    if (!sp->s1_ready) {
        if ((st = s1_upload_padded(sp, &sp->d_eps, sp->eps_host)) != KMX_OK) return st;
        if ((st = s1_upload_padded(sp, &sp->d_mu, sp->mu_host)) != KMX_OK) return st;
        if ((st = s1_build_precond(sp)) != KMX_OK) return st;
        sp->s1_ready = 1;
    }
    if (sp->metric_mode == 0 && !sp->d_metric1) {
        std::vector<double> m1;
        if ((st = build_metric(sp, &m1, 1)) != KMX_OK) return fail(st, "det DF <= 0 at a quadrature point");
        if ((st = upload(&sp->d_metric1, m1)) != KMX_OK) return st;
    }
    if (!sp->h_rr) {
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&sp->h_rr), 2 * sizeof(double), hipHostMallocDefault));
        for (int k = 0; k < 2; ++k) HIP_TRY(hipEventCreateWithFlags(&sp->s1_ev[k], hipEventDisableTiming));
    }
    if (!sp->d_s1) {
        const size_t n = size_t(S1_VECS) * size_t(std::max(sp->n_e, sp->n_h));
        if (hipMalloc(&sp->d_s1, n * sizeof(double)) != hipSuccess)
            return fail(KMX_E_OOM, "device allocation failed (first-scheme vectors)");
        HIP_TRY(hipMemset(sp->d_s1, 0, n * sizeof(double)));
    }
    return KMX_OK;
}

// out = (accumulate ? out : 0) + alpha * (F_z (x) F_y (x) F_x) in, component by
// component, with the dense factors at base + off[c][axis]; `layout`
// names a space with the dims of in and out.  Uses d_tmp (in must differ).
void dense_kron(kmx_space* sp, int layout, const double* base, const int64_t off[3][3], const double* in,
                double* out, double alpha, int accumulate, hipStream_t s) {
    const int64_t nf = std::max(sp->n_e, sp->n_h);
    DenseArgs a{};
    space_dims(sp, layout, a.dims, a.comp_off);
    a.frag = base;
    for (int c = 0; c < 3; ++c)
        for (int ax = 0; ax < 3; ++ax) a.frag_off[c][ax] = off[c][ax];
    ProfScope ps(sp, s, PK_DENSE);
    a.in = in;
    a.in_stride = nf;
    a.out = sp->d_tmp;
    a.out_stride = nf;
    launch_dense_xy(a, 1, s);
    a.in = sp->d_tmp;
    a.out = out;
    a.out_stride = nf;
    a.alpha = alpha;
    a.accumulate = accumulate;
    launch_dense_z(a, 1, s);
}

// y = M x for a 1-form space (SP_E: M^1_eps, SP_H: M~^1_mu)
void run_mass1(kmx_space* sp, int space, const double* x, double* y, hipStream_t s) {
    run_mass(sp, space, false, x, 0, 1, s);
    GatherArgs g{};
    g.patch = sp->d_patch;
    g.patch_stride = sp->patch_per_field;
    patch_size(sp->p, space, sp->ntile, g.patch_comp_off);
    space_dims(sp, space, g.dims, g.comp_off);
    g.ntile = sp->ntile;
    g.out = y;
    g.out_stride = 0;
    ProfScope ps(sp, s, PK_GATHER);
    launch_gather(sp->p, space, g, space == SP_E ? sp->n_e : sp->n_h, 1, s);
}

// z = P^{-1} r with P the separable (Kronecker) approximation of the 1-form mass
void s1_precond(kmx_space* sp, int space, const double* r, double* z, hipStream_t s) {
    dense_kron(sp, space, sp->d_frag_pre, sp->frag_pre_off[space == SP_E ? 0 : 1], r, z, 1.0, 0, s);
}

// y = K~1^T D^1 e (space SP_H) or K1^T D~^1 h (space SP_E): the right-hand
// sides of the (e, h) form, K~1^T block c = G^ along c (x) M^ across and
// K1^T block c = M^T along c (x) G^T across
void s1_rhs(kmx_space* sp, int space, const double* x, double* y, hipStream_t s) {
    double* cu = s1_vec(sp, S1_CU);
    run_curl(sp, space == SP_H, x, 0, cu, 0, 1.0, 0.0, 1, s);
    int64_t off[3][3];
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 3; ++a)
            off[c][a] = sp->frag64_off[FR_PAIR + (space == SP_H ? (a == c ? F_G : F_M) : (a == c ? F_MT : F_GT))];
    dense_kron(sp, space, sp->d_frag64, off, cu, y, 1.0, 0, s);
}

// d_scal[slot] = x . y (deterministic two-level sum)
void s1_dot(kmx_space* sp, const double* x, const double* y, int64_t n, int slot, hipStream_t s) {
    const int nb = energy_blocks(sp);
    ProfScope ps(sp, s, PK_VEC);
    launch_dot(x, y, n, n, 1, sp->d_red, nb, s);
    launch_sum_final(sp->d_red, nb, 1, sp->d_scal + slot, s);
}

// x = M^{-1} y by preconditioned CG from the initial guess in x, to
// |r| <= tol |y|.  The residual norm of every iteration is copied to pinned
// host memory behind an event; the host tests iteration k's norm after it has
// enqueued iteration k + 1, so the device never waits for the host and at most
// one iteration more than needed is run (it only improves x).
kmx_status s1_pcg(kmx_space* sp, int space, const double* y, double* x, double tol, int max_iter,
                  int* iters, hipStream_t s) {
    const int64_t n = space == SP_E ? sp->n_e : sp->n_h;
    double *r = s1_vec(sp, S1_R), *z = s1_vec(sp, S1_Z), *pd = s1_vec(sp, S1_P), *Ap = s1_vec(sp, S1_AP);
    double* sc = sp->d_scal;  // [0], [2] r.z (alternating)  [1] p.Ap  [3] r.r  [4] y.y
    run_mass1(sp, space, x, Ap, s);
    HIP_TRY(hipMemcpyAsync(r, y, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    {
        ProfScope ps(sp, s, PK_VEC);
        launch_axpby(Ap, r, n, -1.0, nullptr, 1.0, s);
    }
    s1_dot(sp, y, y, n, 4, s);
    s1_dot(sp, r, r, n, 3, s);
    double h2[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(h2, sc + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *iters = 0;
    if (!std::isfinite(h2[0]) || !std::isfinite(h2[1])) return fail(KMX_E_UNSTABLE, "mass solve: non-finite input");
    if (h2[1] == 0.0) {  // y = 0: x = 0
        HIP_TRY(hipMemsetAsync(x, 0, n * sizeof(double), s));
        return KMX_OK;
    }
    const double stop = tol * tol * h2[1];
    if (h2[0] <= stop) return KMX_OK;
    s1_precond(sp, space, r, z, s);
    HIP_TRY(hipMemcpyAsync(pd, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    s1_dot(sp, r, z, n, 0, s);
    // r.z alternates between slots 0 and 2 so that no copy is needed
    const int nb = energy_blocks(sp);
    int cur = 0;
    int it = 0;
    // the residual norm of iteration k lands in h_rr[k % 2], marked by s1_ev[k % 2]
    auto converged = [&](int k, bool* done) -> kmx_status {
        HIP_TRY(hipEventSynchronize(sp->s1_ev[k & 1]));
        const double rr = sp->h_rr[k & 1];
        if (!std::isfinite(rr)) return fail(KMX_E_UNSTABLE, "mass solve diverged");
        *done = rr <= stop;
        return KMX_OK;
    };
    bool done = false;
    while (true) {
        run_mass1(sp, space, pd, Ap, s);
        s1_dot(sp, pd, Ap, n, 1, s);
        const int nxt = 2 - cur;
        {
            ProfScope ps(sp, s, PK_VEC);
            launch_cg2(x, r, pd, Ap, nullptr, n, sc + cur, sc + 1, 0, s);
        }
        ++it;
        s1_precond(sp, space, r, z, s);
        {
            ProfScope ps(sp, s, PK_VEC);
            launch_dot2(r, z, n, sp->d_red, nb, sc + 3, sc + nxt, s);
        }
        HIP_TRY(hipMemcpyAsync(sp->h_rr + (it & 1), sc + 3, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(sp->s1_ev[it & 1], s));
        {
            ProfScope ps(sp, s, PK_VEC);
            launch_cg2(x, r, pd, Ap, z, n, sc + nxt, sc + cur, 1, s);
        }
        cur = nxt;
        // test the previous iteration while this one runs
        if (it >= 2) {
            kmx_status st = converged(it - 1, &done);
            if (st != KMX_OK) return st;
            if (done) break;
        }
        if (it >= max_iter) {
            kmx_status st = converged(it, &done);
            if (st != KMX_OK) return st;
            if (done) break;
            *iters = it;
            return fail(KMX_E_UNSTABLE, "mass solve did not reach the tolerance within max_iter iterations");
        }
    }
    *iters = it;
    return KMX_OK;
}

// The same CG with a fixed number of iterations and no read-back (graph
// capture): x = M^{-1} y after `iters` iterations from the guess in x.
void s1_pcg_fixed(kmx_space* sp, int space, const double* y, double* x, int iters, hipStream_t s) {
    const int64_t n = space == SP_E ? sp->n_e : sp->n_h;
    double *r = s1_vec(sp, S1_R), *z = s1_vec(sp, S1_Z), *pd = s1_vec(sp, S1_P), *Ap = s1_vec(sp, S1_AP);
    double* sc = sp->d_scal;
    const int nb = energy_blocks(sp);
    run_mass1(sp, space, x, Ap, s);
    (void)hipMemcpyAsync(r, y, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    launch_axpby(Ap, r, n, -1.0, nullptr, 1.0, s);
    s1_precond(sp, space, r, z, s);
    (void)hipMemcpyAsync(pd, z, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    s1_dot(sp, r, z, n, 0, s);
    int cur = 0;
    for (int it = 0; it < iters; ++it) {
        run_mass1(sp, space, pd, Ap, s);
        s1_dot(sp, pd, Ap, n, 1, s);
        const int nxt = 2 - cur;
        launch_cg2(x, r, pd, Ap, nullptr, n, sc + cur, sc + 1, 0, s);
        s1_precond(sp, space, r, z, s);
        launch_dot2(r, z, n, sp->d_red, nb, sc + 3, sc + nxt, s);
        launch_cg2(x, r, pd, Ap, z, n, sc + nxt, sc + cur, 1, s);
        cur = nxt;
    }
}

// out += alpha * M^{-1} rhs(x) for one half step; the solve starts from the
// previous solution of the same space
kmx_status s1_half(kmx_space* sp, int space, const double* x, double* out, double alpha, double tol, int max_iter,
                   int* iters, hipStream_t s) {
    const int64_t n = space == SP_E ? sp->n_e : sp->n_h;
    double* y = s1_vec(sp, S1_Y);
    double* sol = s1_vec(sp, space == SP_E ? S1_XE : S1_XH);
    s1_rhs(sp, space, x, y, s);
    int it = 0;
    kmx_status st = s1_pcg(sp, space, y, sol, tol, max_iter, &it, s);
    *iters += it;
    if (st != KMX_OK) return st;
    ProfScope ps(sp, s, PK_VEC);
    launch_axpby(sol, out, n, alpha, nullptr, 1.0, s);
    return KMX_OK;
}

kmx_status s1_check(kmx_space* sp, double tol, int max_iter) {
    if (!sp) return fail(KMX_E_ARG, "space is NULL");
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(KMX_E_ARG, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(KMX_E_ARG, "max_iter must be >= 1");
    if (sp->precision == KMX_MIXED) return fail(KMX_E_STATE, "the first scheme runs in FP64 spaces only");
    if (sp->lift_n) return fail(KMX_E_STATE, "the first scheme does not take a lifting");
    return s1_prepare(sp);
}

}  // namespace

extern "C" {

kmx_status kmx_op_mass1(kmx_space* sp, int which, const double* x, double* y, void* stream) {
    if (!sp || !x || !y || (which != 0 && which != 1)) return fail(KMX_E_ARG, "bad argument");
    kmx_status st = s1_prepare(sp);
    if (st != KMX_OK) return st;
    run_mass1(sp, which == 0 ? SP_E : SP_H, x, y, static_cast<hipStream_t>(stream));
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_solve_mass1(kmx_space* sp, int which, const double* y, double* x, double tol, int max_iter,
                           int* iters, void* stream) {
    if (!y || !x || (which != 0 && which != 1)) return fail(KMX_E_ARG, "bad argument");
    kmx_status st = s1_check(sp, tol, max_iter);
    if (st != KMX_OK) return st;
    if (x == y) return fail(KMX_E_ARG, "x and y must not alias");
    int it = 0;
    st = s1_pcg(sp, which == 0 ? SP_E : SP_H, y, x, tol, max_iter, &it, static_cast<hipStream_t>(stream));
    if (iters) *iters = it;
    if (st != KMX_OK) return st;
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_half_step_scheme1(kmx_space* sp, int which, const double* x, double* out, double alpha, double tol,
                                 int max_iter, int* iters, void* stream) {
    if (!x || !out || (which != 0 && which != 1)) return fail(KMX_E_ARG, "bad argument");
    kmx_status st = s1_check(sp, tol, max_iter);
    if (st != KMX_OK) return st;
    int it = 0;
    st = s1_half(sp, which == 0 ? SP_E : SP_H, x, out, alpha, tol, max_iter, &it, static_cast<hipStream_t>(stream));
    if (iters) *iters = it;
    if (st != KMX_OK) return st;
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_project_E1(kmx_space* sp, const double* E_qp_host, double* e_dev, double tol, void* stream) {
    if (!E_qp_host || !e_dev) return fail(KMX_E_ARG, "NULL argument");
    kmx_status st = s1_check(sp, tol, 2000);
    if (st != KMX_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<double> l;
    load_E(sp, E_qp_host, l, 1);
    double* y = s1_vec(sp, S1_Y);
    HIP_TRY(hipMemcpyAsync(y, l.data(), l.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(e_dev, 0, l.size() * sizeof(double), s));
    int it = 0;
    st = s1_pcg(sp, SP_E, y, e_dev, tol, 2000, &it, s);
    if (st != KMX_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));
    return KMX_OK;
}

kmx_status kmx_step_scheme1(kmx_space* sp, double* e, double* h, double dt, int nsteps, double tol, int max_iter,
                            int* iters, void* stream) {
    if (!e || !h) return fail(KMX_E_ARG, "NULL field");
    if (nsteps < 0) return fail(KMX_E_ARG, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return fail(KMX_E_ARG, "dt must be finite");
    kmx_status st = s1_check(sp, tol, max_iter);
    if (st == KMX_OK && sp->dt_cfl1 > 0.0 && std::fabs(dt) > sp->dt_cfl1)
        st = fail(KMX_E_UNSTABLE, "|dt| above the first scheme's CFL limit");
    if (st != KMX_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int it[2] = {0, 0};
    for (int n = 0; n < nsteps && st == KMX_OK; ++n) {
        st = s1_half(sp, SP_H, e, h, -dt, tol, max_iter, &it[1], s);
        if (st == KMX_OK) st = s1_half(sp, SP_E, h, e, dt, tol, max_iter, &it[0], s);
    }
    if (iters) {
        iters[0] = it[0];
        iters[1] = it[1];
    }
    if (st != KMX_OK) return st;
    CHECK_LAUNCH();
    return KMX_OK;
}

kmx_status kmx_graph_create_scheme1(kmx_space* sp, double* e, double* h, double dt, int nsteps, int iters_e,
                                    int iters_h, kmx_graph** out) {
    if (!e || !h || !out || nsteps < 1 || iters_e < 1 || iters_h < 1) return fail(KMX_E_ARG, "bad argument");
    if (!std::isfinite(dt)) return fail(KMX_E_ARG, "dt must be finite");
    kmx_status st = s1_check(sp, 0.5, 1);  // set-up (allocations) before the capture
    if (st != KMX_OK) return st;
    if (sp->dt_cfl1 > 0.0 && std::fabs(dt) > sp->dt_cfl1)
        return fail(KMX_E_UNSTABLE, "|dt| above the first scheme's CFL limit");
    if (sp->prof_on) return fail(KMX_E_STATE, "profiling is on; graphs are captured without timing events");
    *out = nullptr;
    if (!sp->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&sp->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = sp->capture_stream;
    HIP_TRY(hipStreamSynchronize(cs));
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    double* y = s1_vec(sp, S1_Y);
    for (int n = 0; n < nsteps; ++n) {
        // h -= dt M~^{-1} K~1^T D^1 e, then e += dt M^{-1} K1^T D~^1 h
        s1_rhs(sp, SP_H, e, y, cs);
        s1_pcg_fixed(sp, SP_H, y, s1_vec(sp, S1_XH), iters_h, cs);
        launch_axpby(s1_vec(sp, S1_XH), h, sp->n_h, -dt, nullptr, 1.0, cs);
        s1_rhs(sp, SP_E, h, y, cs);
        s1_pcg_fixed(sp, SP_E, y, s1_vec(sp, S1_XE), iters_e, cs);
        launch_axpby(s1_vec(sp, S1_XE), e, sp->n_e, dt, nullptr, 1.0, cs);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (ec != hipSuccess) return fail(KMX_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        hipGraphDestroy(graph);
        return fail(KMX_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    kmx_graph* g = new kmx_graph();
    ++sp->live_graphs;
    g->sp = sp;
    g->graph = graph;
    g->exec = exec;
    g->nsteps = nsteps;
    *out = g;
    return KMX_OK;
}

kmx_status kmx_cfl_scheme1(kmx_space* sp, int max_iter, double tol, double cg_tol, double* dt_max) {
    if (!dt_max || max_iter < 1) return fail(KMX_E_ARG, "bad argument");
    kmx_status st = s1_check(sp, cg_tol, 1000);
    if (st != KMX_OK) return st;
    hipStream_t s = nullptr;
    const int64_t ne = sp->n_e, nh = sp->n_h;
    double *x = nullptr, *hb = nullptr;
    if (hipMalloc(&x, ne * sizeof(double)) != hipSuccess || hipMalloc(&hb, nh * sizeof(double)) != hipSuccess) {
        hipFree(x); hipFree(hb);
        return fail(KMX_E_OOM, "device allocation failed (CFL vectors)");
    }
    // the same seeded start vector as kmx_cfl
    std::vector<double> x0(ne);
    uint64_t rs = 0x9E3779B97F4A7C15ull;
    double nrm = 0.0;
    for (int64_t i = 0; i < ne; ++i) {
        rs = rs * 6364136223846793005ull + 1442695040888963407ull;
        x0[i] = double(rs >> 11) / double(1ull << 53) - 0.5;
        nrm += x0[i] * x0[i];
    }
    for (auto& v : x0) v /= std::sqrt(nrm);
    hipMemcpy(x, x0.data(), ne * sizeof(double), hipMemcpyHostToDevice);
    const int nb = energy_blocks(sp);
    double lam = 0.0;
    int it_cg = 0;
    for (int it = 0; it < max_iter && st == KMX_OK; ++it) {
        // x <- A1 x = M^{-1} K1^T D~^1 M~^{-1} K~1^T D^1 x, then normalised
        hipMemsetAsync(hb, 0, nh * sizeof(double), s);
        st = s1_half(sp, SP_H, x, hb, 1.0, cg_tol, 1000, &it_cg, s);
        if (st != KMX_OK) break;
        hipMemsetAsync(x, 0, ne * sizeof(double), s);
        st = s1_half(sp, SP_E, hb, x, 1.0, cg_tol, 1000, &it_cg, s);
        if (st != KMX_OK) break;
        launch_dot(x, x, ne, ne, 1, sp->d_red, nb, s);
        launch_sum_final(sp->d_red, nb, 1, sp->d_scal + 8, s);
        double yy = 0.0;
        hipMemcpy(&yy, sp->d_scal + 8, sizeof(double), hipMemcpyDeviceToHost);
        const double lam_new = std::sqrt(yy);
        if (!std::isfinite(lam_new) || lam_new <= 0.0) { st = fail(KMX_E_UNSTABLE, "power iteration failed"); break; }
        launch_axpby(x, x, ne, 1.0 / lam_new, nullptr, 0.0, s);
        const bool done = std::fabs(lam_new - lam) <= tol * lam_new;
        lam = lam_new;
        if (done) break;
    }
    hipDeviceSynchronize();
    hipFree(x);
    hipFree(hb);
    if (st != KMX_OK) return st;
    *dt_max = 2.0 / std::sqrt(lam);
    sp->dt_cfl1 = *dt_max;
    return KMX_OK;
}

}  // extern "C"
