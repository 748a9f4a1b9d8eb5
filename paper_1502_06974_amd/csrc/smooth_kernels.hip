// Time/frequency smoothing of the scalar StefCal update (Sect. 3.4).  Each sample of an
// interval is a cell (t, nu) of an n_time x n_chan grid (sample s = t * n_chan + nu) with
// gains of its own.  With alpha_p(t, nu) = sum_q conj(y) d and beta_p(t, nu) = sum_q |y|^2
// (the per-antenna sums of Eqs. JHJ:DI:tfw, JHR:DI:tfw without the sum over samples, y formed
// with the gains of the row's own cell), every update takes
//     g_p(t, nu) = (w o alpha_p)(t, nu) / (w o beta_p)(t, nu)              (Eq. JHJ:diag:smooth)
// for a Gaussian w of widths sigma_t, sigma_f cells truncated at three widths (cells beyond
// the grid edge are absent from both sums), then the schedule of Sect. 3.1.
//
// The per-cell sums come from the scalar pass run over a cell plan: the same rows, every
// cell an interval of one sample (so the triangle pass applies to canonical tables).  Then
// per update: fold of each cell's tile partials, a frequency then a time pass of the
// separable convolution (FP64 accumulation), the per-cell ratio and schedule written in
// place, and one workgroup per interval (a chunk of cells) that takes the decision.
// Convergence: the relative change over the chunk's cells and antennas after removing, per
// cell, the best phase between the iterates (each cell's solution answers its own weighted
// least-squares problem, Eq. cal:DI:smooth, defined up to one phase per cell), from
// ||g_new e^{-i phi} - g_old||^2 = ||g_new||^2 + ||g_old||^2 - 2 |S|, S = sum conj(g_old) g_new
// over the cell's antennas, in FP64.  With noise the smoothed iterates keep turning along
// these phases, which the plain relative change would never see stop.
#include <cmath>
#include <utility>
#include <vector>

#include "di_common.h"

using namespace wcal_dev;

struct SmoothPlan {
    wcal_plan* cells = nullptr;   // every sample of every interval as an interval of its own
    int32_t nt = 0, nf = 0;       // grid of one interval
    int32_t rt = 0, rf = 0;       // kernel radii (ceil(3 sigma); 0 for sigma = 0)
    float* d_ab = nullptr;        // [cells][n_ant][3] beta, Re alpha, Im alpha; smoothed in place
    float* d_tmp = nullptr;       // [cells][n_ant][3] after the frequency pass
    double* d_part = nullptr;     // [n_int][bpc][2] |g_new|^2 and the phase-aligned change per block
    int32_t* d_flag = nullptr;    // [n_int] 1: non-finite sums, 2: a singular cell (this update)
    int32_t* d_active = nullptr;  // [n_int]
    float* d_taps = nullptr;      // w_t(0..rt), then w_f(0..rf) (a table: plan-owned)
    int32_t cpb = 0, bpc = 0;     // update: cells per workgroup, workgroups per interval
    int32_t n_int = 0, n_ant = 0;
    // workspace: the five scratch arrays above, then the cell plan's workspace
    size_t off[6] = {};
};

namespace {

constexpr int SB = 256;

__global__ void __launch_bounds__(SB) sm_init_kernel(int n_int, uint32_t* status, int32_t* n_iter,
                                                     int32_t* active, int32_t* flag, int32_t* ctr, int nctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_int) {
        status[i] = 0;
        n_iter[i] = 0;
        active[i] = 1;
        flag[i] = 0;
    }
    if (i < nctr) ctr[i] = 0;
}

// ab[c][p][j] = sum over the tiles of cell c (in tile order) of the pass partials
__global__ void __launch_bounds__(SB) sm_fold_kernel(const float* __restrict__ partial, const int32_t* __restrict__ toff,
                                                     int64_t n, int na, int ncell, const int32_t* active,
                                                     int32_t* flag, float* __restrict__ ab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = i / (3 * na);
    const int k = (int)(c / ncell);
    if (!active[k]) return;
    const int r = (int)(i % (3 * na));
    float v = 0.f;
    for (int t = toff[c]; t < toff[c + 1]; ++t) v += partial[(int64_t)t * na * 3 + r];
    ab[i] = v;
    if (!isfinite(v)) atomicOr(&flag[k], 1);
}

// One axis of the separable convolution: out[x] = sum_j w(|j|) in[x + j * stride] over the
// cells of the grid line through x (axis length len, position pos of x on it).
__global__ void __launch_bounds__(SB) sm_conv_kernel(const float* __restrict__ in, float* __restrict__ out, int64_t n,
                                                     int na, int ncell, int nf, int along_t, int r,
                                                     const float* __restrict__ taps, const int32_t* active) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = i / (3 * na);
    const int k = (int)(c / ncell);
    if (!active[k]) return;
    const int cl = (int)(c % ncell);
    const int pos = along_t ? cl / nf : cl % nf;
    const int len = along_t ? ncell / nf : nf;
    const int64_t stride = (int64_t)(along_t ? nf : 1) * 3 * na;
    const int j0 = max(-r, -pos), j1 = min(r, len - 1 - pos);
    double acc = 0.0;
    for (int j = j0; j <= j1; ++j) acc += (double)taps[j < 0 ? -j : j] * (double)in[i + j * stride];
    out[i] = (float)acc;
}

// The same one-axis pass through LDS: a workgroup owns CT_C consecutive cells of one line of
// the grid (a time slot along frequency, or a channel along time) and CT_E consecutive
// (antenna, component) values, loads them with the kernel's halo once, and sums the taps
// in the order of sm_conv_kernel (so the results are the same bits).  Radii up to CT_RMAX.
constexpr int CT_C = 64;
constexpr int CT_E = 64;
constexpr int CT_RMAX = 64;
__global__ void __launch_bounds__(SB) sm_conv_tile_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                          int na, int ncell, int nf, int along_t, int r,
                                                          const float* __restrict__ taps,
                                                          const int32_t* active, int ntc, int nte, int nline) {
    __shared__ float sh[(CT_C + 2 * CT_RMAX) * CT_E];
    __shared__ float stap[CT_RMAX + 1];
    int b = blockIdx.x;
    const int te = b % nte;
    b /= nte;
    const int tc = b % ntc;
    b /= ntc;
    const int line = b % nline, k = b / nline;
    if (!active[k]) return;
    const int E = 3 * na;
    const int len = along_t ? ncell / nf : nf;
    const int64_t S = (int64_t)(along_t ? nf : 1) * E;
    const int64_t base = ((int64_t)k * ncell + (along_t ? line : (int64_t)line * nf)) * E;
    const int p0 = tc * CT_C, e0 = te * CT_E;
    const int lo = max(0, p0 - r), hi = min(len, p0 + CT_C + r);   // cells loaded: [lo, hi)
    const int ne = min(CT_E, E - e0);
    for (int i = threadIdx.x; i <= r; i += SB) stap[i] = taps[i];
    for (int i = threadIdx.x; i < (hi - lo) * CT_E; i += SB) {
        const int pc = i / CT_E, e = i - pc * CT_E;
        if (e < ne) sh[i] = in[base + (int64_t)(lo + pc) * S + e0 + e];
    }
    __syncthreads();
    const int np = min(CT_C, len - p0);
    for (int i = threadIdx.x; i < np * CT_E; i += SB) {
        const int pc = i / CT_E, e = i - pc * CT_E;
        if (e >= ne) continue;
        const int pos = p0 + pc;
        const int j0 = max(-r, -pos), j1 = min(r, len - 1 - pos);
        double acc = 0.0;
        for (int j = j0; j <= j1; ++j) acc += (double)stap[j < 0 ? -j : j] * (double)sh[(pos + j - lo) * CT_E + e];
        out[base + (int64_t)pos * S + e0 + e] = (float)acc;
    }
}

// Per (cell, antenna) of a chunk: the smoothed GN value, the schedule, the gains written in
// place (unless the chunk's sums are not finite).  A workgroup owns cpb whole cells of one
// chunk (cpb = SB / n_ant, or one cell with threads striding over the antennas when
// n_ant > SB); per cell it forms |g_new|^2, |g_old|^2 and S = sum conj(g_old) g_new over the
// antennas in a fixed order, the per-cell phase-aligned change |g_new|^2 + |g_old|^2 - 2|S|,
// and writes the workgroup's FP64 sums of |g_new|^2 and of that change.
__global__ void __launch_bounds__(SB) sm_update_kernel(const float* __restrict__ ab, float2* __restrict__ gains,
                                                       int na, int ncell, int cpb, int bpc, int schedule, int it,
                                                       const int32_t* active, int32_t* flag, double* part) {
    __shared__ double red[SB / WAVE];
    __shared__ double t_an[SB], t_bo[SB], t_sr[SB], t_si[SB];
    const int k = blockIdx.x / bpc, j = blockIdx.x % bpc;
    if (!active[k]) return;
    const bool bad = (flag[k] & 1) != 0;
    const bool avg = avg_step(it, schedule);
    const int c0 = j * cpb, nc = min(cpb, ncell - c0);
    double an = 0.0, bo = 0.0, sr = 0.0, si = 0.0;
    for (int e = threadIdx.x; e < nc * na; e += SB) {
        const int64_t i = ((int64_t)k * ncell + c0) * na + e;     // (cell, antenna)
        const double beta = ab[3 * i], ar = ab[3 * i + 1], ai = ab[3 * i + 2];
        const float2 go = gains[i];
        double gr = go.x, gi = go.y;
        if (beta > 0.0) { gr = ar / beta; gi = ai / beta; }
        else atomicOr(&flag[k], 2);
        if (avg) { gr = 0.5 * (go.x + gr); gi = 0.5 * (go.y + gi); }
        const float2 g = make_float2((float)gr, (float)gi);
        if (!bad) gains[i] = g;
        an += (double)g.x * g.x + (double)g.y * g.y;
        bo += (double)go.x * go.x + (double)go.y * go.y;
        sr += (double)go.x * g.x + (double)go.y * g.y;        // conj(g_old) g_new
        si += (double)go.x * g.y - (double)go.y * g.x;
    }
    double cell_a = 0.0, cell_d = 0.0;
    if (cpb == 1) {
        an = block_sum(an, red);
        bo = block_sum(bo, red);
        sr = block_sum(sr, red);
        si = block_sum(si, red);
        cell_a = an;
        cell_d = fmax(an + bo - 2.0 * sqrt(sr * sr + si * si), 0.0);
    } else {
        // one (cell, antenna) per thread: each cell's antennas summed in order by one thread
        t_an[threadIdx.x] = an; t_bo[threadIdx.x] = bo; t_sr[threadIdx.x] = sr; t_si[threadIdx.x] = si;
        __syncthreads();
        double a_ = 0.0, d_ = 0.0;
        if ((int)threadIdx.x < nc) {
            double xa = 0.0, xb = 0.0, xr = 0.0, xi = 0.0;
            for (int p = 0; p < na; ++p) {
                const int e = threadIdx.x * na + p;
                xa += t_an[e]; xb += t_bo[e]; xr += t_sr[e]; xi += t_si[e];
            }
            a_ = xa;
            d_ = fmax(xa + xb - 2.0 * sqrt(xr * xr + xi * xi), 0.0);
        }
        cell_a = block_sum(a_, red);
        cell_d = block_sum(d_, red);
    }
    if (threadIdx.x == 0) {
        double* q = part + ((int64_t)k * bpc + j) * 2;
        q[0] = cell_a;
        q[1] = cell_d;
    }
}

// One workgroup per interval: the decision of update `it` and, if the interval keeps
// iterating, the tiles of its cells listed for the next pass of the cell plan.
__global__ void __launch_bounds__(SB) sm_finish_kernel(const double* part, int bpc, int32_t* flag, int32_t* active,
                                                       uint32_t* status, int32_t* n_iter, int it, int max_iter,
                                                       double tol, int ncell, const int32_t* toff, int32_t* lists,
                                                       int ntiles, int32_t* ctr, int qoff) {
    __shared__ double red[SB / WAVE];
    __shared__ int s_pos;
    const int k = blockIdx.x;
    if (!active[k]) return;
    double an = 0.0, dd = 0.0;
    for (int j = threadIdx.x; j < bpc; j += blockDim.x) {
        const double* q = part + ((int64_t)k * bpc + j) * 2;
        an += q[0]; dd += q[1];
    }
    an = block_sum(an, red);
    dd = block_sum(dd, red);
    const int f = flag[k];
    uint32_t st = 0;
    bool finished = false;
    if (f & 1) {
        st |= WCAL_NONFINITE;
        finished = true;
    } else {
        if (f & 2) st |= WCAL_SINGULAR_ANT;
        const double rel = an == 0.0 ? (dd == 0.0 ? 0.0 : INFINITY) : sqrt(dd / an);
        if (rel < tol) { st |= WCAL_CONVERGED; finished = true; }
    }
    if (!finished && it + 1 >= max_iter) {
        st |= WCAL_MAXITER;
        finished = true;
    }
    const int t0 = toff[(int64_t)k * ncell], t1 = toff[(int64_t)(k + 1) * ncell];
    __syncthreads();     // every thread has read flag[k]
    if (threadIdx.x == 0) {
        status[k] |= st;
        if (!(st & WCAL_NONFINITE)) n_iter[k] = it + 1;
        flag[k] = 0;
        if (finished) active[k] = 0;
        else s_pos = atomicAdd(&ctr[qoff + it + 1], t1 - t0);
    }
    if (!finished) {
        __syncthreads();
        int32_t* next = lists + ((it + 1) & 1) * ntiles;
        for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) next[s_pos + i] = t0 + i;
    }
}

// chi^2 per interval from the residual tiles of its cells: one workgroup per interval, each
// thread a fixed strided share of the tiles, then the fixed-order workgroup sum
__global__ void __launch_bounds__(SB) sm_chi2_kernel(const double* chi_part, const int32_t* toff, int ncell,
                                                     double* chi2) {
    __shared__ double red[SB / WAVE];
    const int k = blockIdx.x;
    double c = 0.0;
    for (int t = toff[(int64_t)k * ncell] + threadIdx.x; t < toff[(int64_t)(k + 1) * ncell]; t += SB)
        c += chi_part[t];
    c = block_sum(c, red);
    if (threadIdx.x == 0) chi2[k] = c;
}

unsigned nblk(int64_t n) { return (unsigned)((n + SB - 1) / SB); }

}  // namespace

void smooth_free(SmoothPlan* sp) {
    if (!sp) return;
    wcal_plan_destroy(sp->cells);
    if (sp->d_taps) (void)hipFree(sp->d_taps);
    delete sp;
}

// Workspace of the smoothing scratch: the per-cell sums and their convolution, the per-block
// norms, the per-interval flags and activity, then the cell plan's own workspace.
static void smooth_layout(SmoothPlan* sp) {
    const size_t ncells = (size_t)sp->cells->prob.n_int;
    const size_t nab = ncells * sp->n_ant * 3;
    const size_t sz[5] = {nab * sizeof(float), nab * sizeof(float), (size_t)sp->n_int * sp->bpc * 2 * sizeof(double),
                          (size_t)sp->n_int * sizeof(int32_t), (size_t)sp->n_int * sizeof(int32_t)};
    sp->off[0] = 0;
    for (int i = 0; i < 5; ++i) sp->off[i + 1] = sp->off[i] + ws_round(sz[i]);
}

size_t smooth_ws_bytes(const SmoothPlan* sp) { return sp->off[5] + sp->cells->ws_bytes; }

void smooth_ws_bind(SmoothPlan* sp, char* ws) {
    sp->d_ab = reinterpret_cast<float*>(ws + sp->off[0]);
    sp->d_tmp = reinterpret_cast<float*>(ws + sp->off[1]);
    sp->d_part = reinterpret_cast<double*>(ws + sp->off[2]);
    sp->d_flag = reinterpret_cast<int32_t*>(ws + sp->off[3]);
    sp->d_active = reinterpret_cast<int32_t*>(ws + sp->off[4]);
    ws_bind(sp->cells, ws + sp->off[5]);
}

extern "C" {

int wcal_plan_smoothing(wcal_plan* plan, int32_t n_time, int32_t n_chan, double sigma_t, double sigma_f) {
    if (!plan) return wcal_error(WCAL_EINVAL, "NULL plan");
    const wcal_problem& p = plan->prob;
    if (p.algo != WCAL_STEFCAL || p.n_corr != 1 || p.n_dir != 1)
        return wcal_error(WCAL_EINVAL, "smoothing is implemented for scalar StefCal");
    if (p.mode != WCAL_MODE_PASS) return wcal_error(WCAL_EINVAL, "smoothing needs PASS mode");
    if (n_time < 1 || n_chan < 1 || !(sigma_t >= 0.0) || !(sigma_f >= 0.0) || !std::isfinite(sigma_t) ||
        !std::isfinite(sigma_f))
        return wcal_error(WCAL_EINVAL, "n_time, n_chan >= 1 and finite sigmas >= 0 required");
    const int64_t ncell = (int64_t)n_time * n_chan;
    for (int32_t k = 0; k < p.n_int; ++k)
        if (plan->h_ns[k] != ncell) return wcal_error(WCAL_ESHAPE, "every interval must hold n_time * n_chan samples");
    const int64_t ncells = ncell * p.n_int;
    if (ncells > INT32_MAX / 2) return wcal_error(WCAL_ESHAPE, "too many cells");
    if (hipSetDevice(plan->device) != hipSuccess) return wcal_error(WCAL_EHIP, "hipSetDevice failed");
    smooth_free(plan->smooth);
    plan->smooth = nullptr;
    auto* sp = new SmoothPlan();
    sp->nt = n_time;
    sp->nf = n_chan;
    sp->rt = sigma_t > 0.0 ? (int)std::ceil(3.0 * sigma_t) : 0;
    sp->rf = sigma_f > 0.0 ? (int)std::ceil(3.0 * sigma_f) : 0;
    if (sp->rt > 4096 || sp->rf > 4096) {
        delete sp;
        return wcal_error(WCAL_ESHAPE, "smoothing width above 1365 cells");
    }
    // the cell plan: same baselines, one sample per interval
    std::vector<int32_t> a1(p.n_bl), a2(p.n_bl);
    if (hipMemcpy(a1.data(), plan->d_ant1, sizeof(int32_t) * p.n_bl, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(a2.data(), plan->d_ant2, sizeof(int32_t) * p.n_bl, hipMemcpyDeviceToHost) != hipSuccess) {
        delete sp;
        return wcal_error(WCAL_EHIP, "reading the baseline table failed");
    }
    wcal_problem cp = p;
    cp.n_int = (int32_t)ncells;
    std::vector<int64_t> ones((size_t)ncells, 1);
    int rc = wcal_plan_create(&cp, a1.data(), a2.data(), ones.data(), plan->device, &sp->cells);
    if (rc != WCAL_OK) {
        delete sp;
        return rc;
    }
    // the cell plan's passes are launched one update at a time (the smoothed update needs the
    // sums of neighbouring cells): no device-side loop
    sp->cells->loop = false;
    // its triangle tiles feed only the unfused pass: packed rows
    sp->cells->tri_unfused = true;
    if (sp->cells->tri && (rc = plan_retile(sp->cells)) != WCAL_OK) {
        smooth_free(sp);
        return rc;
    }
    ws_layout(sp->cells);
    const int na = p.n_ant;
    sp->cpb = na <= SB ? SB / na : 1;
    sp->bpc = (int)((ncell + sp->cpb - 1) / sp->cpb);
    std::vector<float> taps;
    for (int j = 0; j <= sp->rt; ++j) taps.push_back(sp->rt ? (float)std::exp(-0.5 * j * j / (sigma_t * sigma_t)) : 1.f);
    for (int j = 0; j <= sp->rf; ++j) taps.push_back(sp->rf ? (float)std::exp(-0.5 * j * j / (sigma_f * sigma_f)) : 1.f);
    sp->n_int = p.n_int;
    sp->n_ant = na;
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&sp->d_taps), taps.size() * sizeof(float))) != hipSuccess ||
        (e = hipMemcpy(sp->d_taps, taps.data(), taps.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
        smooth_free(sp);
        return wcal_error(e == hipErrorOutOfMemory ? WCAL_ENOMEM : WCAL_EHIP, "smoothing table allocation failed");
    }
    smooth_layout(sp);
    plan->smooth = sp;
    ws_layout(plan);
    return WCAL_OK;
}

int wcal_solve_smooth(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                      wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
                      void* workspace, size_t ws_bytes, void* stream) {
    if (!plan || !data || !model || !gains || !n_iter || !status) return wcal_error(WCAL_EINVAL, "NULL argument");
    SmoothPlan* sp = plan->smooth;
    if (!sp) return wcal_error(WCAL_EINVAL, "call wcal_plan_smoothing first");
    if (reinterpret_cast<uintptr_t>(data) % 8 || reinterpret_cast<uintptr_t>(model) % 8 ||
        reinterpret_cast<uintptr_t>(gains) % 8 || (residual && reinterpret_cast<uintptr_t>(residual) % 8))
        return wcal_error(WCAL_EINVAL, "complex arrays must be 8-byte aligned");
    if (hipSetDevice(plan->device) != hipSuccess) return wcal_error(WCAL_EHIP, "hipSetDevice failed");
    if (int rc = ws_check_bind(plan, workspace, ws_bytes)) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const wcal_plan* cp = sp->cells;
    const wcal_problem& p = plan->prob;
    const int na = p.n_ant, ncell = sp->nt * sp->nf;
    const int64_t nab = (int64_t)cp->prob.n_int * na * 3;
    DiArgs a{};
    fill_di_args(cp, a);
    a.data = reinterpret_cast<const float2*>(data);
    a.model = reinterpret_cast<const float2*>(model);
    a.flags = flags;
    a.gains = reinterpret_cast<float2*>(gains);
    const int nctr = 2 * (cp->prob.max_iter + 2);
    const int32_t* toff = di_pass_tile_off(cp);
    const int32_t npt = di_pass_ntiles(cp);
    prof_begin(plan, WCAL_K_OTHER, s);
    hipLaunchKernelGGL(sm_init_kernel, dim3(nblk(std::max(p.n_int, nctr))), dim3(SB), 0, s, p.n_int, status, n_iter,
                       sp->d_active, sp->d_flag, cp->d_ctr, nctr);
    prof_end(plan, WCAL_K_OTHER, s);
    for (int it = 0; it < p.max_iter; ++it) {
        hipError_t e = launch_di_pass_partials(cp, plan, a, it, s);
        if (e != hipSuccess) return wcal_error(WCAL_EHIP, "smoothed pass launch failed");
        prof_begin(plan, WCAL_K_UPDATE, s);
        hipLaunchKernelGGL(sm_fold_kernel, dim3(nblk(nab)), dim3(SB), 0, s, (const float*)cp->d_partial, toff, nab, na,
                           ncell, (const int32_t*)sp->d_active, sp->d_flag, sp->d_ab);
        // the two one-axis passes; an axis of radius 0 is the identity (its only tap is 1) and
        // is skipped
        float* cur = sp->d_ab;
        float* spare = sp->d_tmp;
        auto conv = [&](int along_t, int r, const float* taps) {
            if (r <= CT_RMAX) {
                const int len = along_t ? ncell / sp->nf : sp->nf;
                const int nline = ncell / len, ntc = (len + CT_C - 1) / CT_C, nte = (3 * na + CT_E - 1) / CT_E;
                hipLaunchKernelGGL(sm_conv_tile_kernel, dim3((unsigned)((int64_t)p.n_int * nline * ntc * nte)), dim3(SB),
                                   0, s, (const float*)cur, spare, na, ncell, sp->nf, along_t, r, taps,
                                   (const int32_t*)sp->d_active, ntc, nte, nline);
            } else {
                hipLaunchKernelGGL(sm_conv_kernel, dim3(nblk(nab)), dim3(SB), 0, s, (const float*)cur, spare, nab, na,
                                   ncell, sp->nf, along_t, r, taps, (const int32_t*)sp->d_active);
            }
            std::swap(cur, spare);
        };
        if (sp->rf > 0) conv(0, sp->rf, (const float*)(sp->d_taps + sp->rt + 1));
        if (sp->rt > 0) conv(1, sp->rt, (const float*)sp->d_taps);
        hipLaunchKernelGGL(sm_update_kernel, dim3((unsigned)(p.n_int * sp->bpc)), dim3(SB), 0, s, (const float*)cur,
                           a.gains, na, ncell, sp->cpb, sp->bpc, p.schedule, it, (const int32_t*)sp->d_active,
                           sp->d_flag, sp->d_part);
        hipLaunchKernelGGL(sm_finish_kernel, dim3(p.n_int), dim3(SB), 0, s, (const double*)sp->d_part, sp->bpc,
                           sp->d_flag, sp->d_active, status, n_iter, it, p.max_iter, p.tol, ncell, toff, cp->d_lists,
                           npt, cp->d_ctr, cp->prob.max_iter + 2);
        prof_end(plan, WCAL_K_UPDATE, s);
        if (watch_stop(plan, s, cp->d_ctr + (cp->prob.max_iter + 2) + it + 1, it)) break;   // tiles listed for it + 1
    }
    if (residual || chi2) {
        DiArgs r = a;
        r.gains_in = a.gains;
        r.residual = reinterpret_cast<float2*>(residual);
        if (launch_di_resid_tiles(cp, plan, r, s) != hipSuccess) return wcal_error(WCAL_EHIP, "residual launch failed");
        if (chi2)
            hipLaunchKernelGGL(sm_chi2_kernel, dim3(p.n_int), dim3(SB), 0, s, (const double*)cp->d_chi_part,
                               (const int32_t*)cp->d_tile_off, ncell, chi2);
    }
    return hipGetLastError() == hipSuccess ? WCAL_OK : wcal_error(WCAL_EHIP, "smoothed solve launch failed");
}

}  // extern "C"
