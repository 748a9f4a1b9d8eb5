// Pieces shared by the direction-dependent solvers (scalar gains in dd_kernels.hip, 2x2
// Jones gains in ddp_kernels.hip): the solve state carved out of the plan's record buffer,
// the work counters, the per-interval decision after an update and launch sizing.
//
// The solve of both is the same loop: a Gram pass writes one record of gain-independent
// sums over samples per (interval, baseline); one workgroup per (interval, antenna)
// contracts the records of the antenna's baselines with the current gains, solves and
// writes the candidate gains and its share of the FP64 relative-change norms;
// dd_finish_kernel decides per interval.
#pragma once

#include "di_common.h"

namespace wcal_dev {

constexpr int DT = 256;          // workgroup size of the direction-dependent kernels

typedef float floatx4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline int ntri(int n) { return n * (n + 1) / 2; }
// packed index of (i, j), i <= j < n, row-major upper triangle
__host__ __device__ inline int tri(int i, int j, int n) { return i * n - i * (i - 1) / 2 + (j - i); }

__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

struct DdState {
    float* rec;          // [n_int][n_bl][record floats]
    double* chi_bl;      // [n_int][n_bl] chi^2 per baseline (accumulate)
    float2* gn;          // [n_int][nd][n_ant][n_corr] candidate gains of the current update
    double* ant_d;       // [n_int][n_ant] |g_new - g|^2 per antenna
    double* ant_n;       // [n_int][n_ant] |g_new|^2 per antenna
    int32_t* ant_f;      // [n_int][n_ant] 1: non-finite block, 2: singular block
    int32_t* alist;      // [2][n_int] intervals still iterating, by update parity
    const int32_t* ant_ptr;  // [n_ant + 1] CSR of (baseline, side) per antenna
    const int32_t* ant_bl;   // [2 n_bl]: 2 b + side (side 0: antenna is ant1, 1: ant2)
    int32_t* active;     // [n_int]
    int32_t* ctr;        // work counters
    const Tile* tiles;
    const int32_t* tile_off;
    int32_t ntiles;
    double* chi_part;    // [ntiles]
};

// Bytes of the state for record size rec_floats (floats per baseline record).
inline size_t dd_state_bytes(const wcal_problem& p, int rec_floats) {
    const size_t n = (size_t)p.n_int * p.n_bl;
    const size_t na = (size_t)p.n_int * p.n_ant;
    return n * rec_floats * sizeof(float) + n * sizeof(double) + 2 * na * sizeof(double) +
           na * p.n_dir * p.n_corr * sizeof(float2) + na * sizeof(int32_t) + 2 * (size_t)p.n_int * sizeof(int32_t);
}

inline DdState dd_state_of(const wcal_plan* plan, int rec_floats) {
    const wcal_problem& p = plan->prob;
    DdState st;
    st.rec = plan->d_stats;
    const size_t nrec = (size_t)p.n_int * p.n_bl;
    st.chi_bl = reinterpret_cast<double*>(plan->d_stats + nrec * rec_floats);
    st.ant_d = st.chi_bl + nrec;
    st.ant_n = st.ant_d + (size_t)p.n_int * p.n_ant;
    st.gn = reinterpret_cast<float2*>(st.ant_n + (size_t)p.n_int * p.n_ant);
    st.ant_f = reinterpret_cast<int32_t*>(st.gn + (size_t)p.n_int * p.n_dir * p.n_ant * p.n_corr);
    st.alist = st.ant_f + (size_t)p.n_int * p.n_ant;
    st.ant_ptr = plan->d_ant_ptr;
    st.ant_bl = plan->d_ant_bl;
    st.active = plan->d_active;
    st.ctr = plan->d_ctr;
    st.tiles = plan->d_tiles;
    st.tile_off = plan->d_tile_off;
    st.ntiles = plan->ntiles;
    st.chi_part = plan->d_chi_part;
    return st;
}

// counters: [0] one-off Gram pops, [2 + 2 it] Gram pops of update it, [3 + 2 it] intervals
// listed for update it (it >= 1)
__host__ __device__ inline int dd_pop_slot(int it) { return 2 + 2 * it; }
__host__ __device__ inline int dd_nlist_slot(int it) { return 3 + 2 * it; }

// Workgroups for a persistent launch: as many as fit on the device at once, at most `work`.
inline int dd_grid(const wcal_plan* plan, const void* fn, size_t smem, int64_t work) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, DT, smem) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t g = (int64_t)per_cu * plan->n_cu;
    if (g > work) g = work;
    return (int)(g < 1 ? 1 : g);
}

namespace {

__global__ void __launch_bounds__(DT) dd_init_kernel(DdArgs a, DdState st, int init_state, int nctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (init_state && i < a.n_int) {
        a.status[i] = 0;
        a.n_iter[i] = 0;
        st.active[i] = 1;
    }
    if (i < nctr) st.ctr[i] = 0;
}

// The interval's decision after the per-antenna update: norms summed over antennas in a
// fixed order; a non-finite block stops the interval before this update (gains kept);
// otherwise the candidate becomes the gains, singular antennas are reported, and the
// relative change and the iteration cap decide whether it keeps iterating.
__global__ void __launch_bounds__(DT) dd_finish_kernel(DdArgs a, DdState st, int it) {
    __shared__ double red[DT / WAVE];
    __shared__ int s_f;
    const int k = blockIdx.x;
    if (!st.active[k]) return;
    const int na = a.n_ant;
    const int per = a.n_dir * na * a.n_corr;
    if (threadIdx.x == 0) s_f = 0;
    __syncthreads();
    double dsum = 0.0, nsum = 0.0;
    int f = 0;
    for (int p = threadIdx.x; p < na; p += blockDim.x) {
        dsum += st.ant_d[(int64_t)k * na + p];
        nsum += st.ant_n[(int64_t)k * na + p];
        f |= st.ant_f[(int64_t)k * na + p];
    }
    if (f) atomicOr(&s_f, f);
    dsum = block_sum(dsum, red);
    nsum = block_sum(nsum, red);
    const int flags = s_f;
    uint32_t status = 0;
    bool finished = false;
    if (flags & 1) {
        status |= WCAL_NONFINITE;
        finished = true;
    } else {
        if (flags & 2) status |= WCAL_SINGULAR_ANT;
        const float2* gn = st.gn + (int64_t)k * per;
        float2* gk = a.gains + (int64_t)k * per;
        for (int i = threadIdx.x; i < per; i += blockDim.x) gk[i] = gn[i];
        const double num = sqrt(dsum), den = sqrt(nsum);
        const double rel = den == 0.0 ? (num == 0.0 ? 0.0 : INFINITY) : num / den;
        if (rel < a.tol) { status |= WCAL_CONVERGED; finished = true; }
    }
    if (!finished && it + 1 >= a.max_iter) {
        status |= WCAL_MAXITER;
        finished = true;
    }
    if (threadIdx.x == 0) {
        a.status[k] |= status;
        if (!(status & WCAL_NONFINITE)) a.n_iter[k] = it + 1;
        if (finished) st.active[k] = 0;
        else st.alist[((it + 1) & 1) * a.n_int + atomicAdd(&st.ctr[dd_nlist_slot(it + 1)], 1)] = k;
    }
}

// chi^2 per interval from the residual tiles' partials, in tile order
__global__ void __launch_bounds__(DT) dd_chi2_kernel(DdArgs a, DdState st) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_int || !a.chi2) return;
    double c = 0.0;
    for (int t = st.tile_off[k]; t < st.tile_off[k + 1]; ++t) c += st.chi_part[t];
    a.chi2[k] = c;
}

}  // namespace

}  // namespace wcal_dev
