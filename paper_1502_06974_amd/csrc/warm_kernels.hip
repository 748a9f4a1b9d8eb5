// Learned warm start, device side.  Single-channel intervals are grouped in bins of
// bin_width consecutive intervals; bin B = [lo, hi) has the knot interval
// lo + (hi - lo - 1) / 2.  The coarse pass solves the knot intervals only (their rows are
// gathered here into a compact batch for a second plan); the network maps the knot gains
// to knot values; those are spread to every interval by interpolating amplitude and phase
// linearly between neighbouring knots.  Training targets are the full solve's gains,
// referenced to antenna 0 (times conj(g_0)/|g_0| per interval, the phase gauge), averaged
// over a window around each knot.  Intervals that do not converge from the warm start are
// reset to unit gains for another solve.
#include "wcal_internal.h"

namespace {

constexpr int WB = 256;

__device__ __host__ inline int knot_of(int B, int bin_width, int n_int) {
    const int lo = B * bin_width;
    const int hi = min(lo + bin_width, n_int);
    return lo + (hi - lo - 1) / 2;
}

// grid.y = bin; each workgroup first finds the bin's output row offset (rows of the knots
// of the bins before it), then copies a strided share of the knot interval's rows.
__global__ void __launch_bounds__(WB) gather_knots_kernel(int n_int, int bin_width, const int64_t* __restrict__ row_off,
                                                          int nc, int nmc, const float2* __restrict__ data,
                                                          const float2* __restrict__ model,
                                                          const uint8_t* __restrict__ flags, float2* __restrict__ data_out,
                                                          float2* __restrict__ model_out, uint8_t* __restrict__ flags_out) {
    __shared__ int64_t red[WB];
    const int B = blockIdx.y;
    int64_t part = 0;
    for (int b = threadIdx.x; b < B; b += WB) {
        const int k = knot_of(b, bin_width, n_int);
        part += row_off[k + 1] - row_off[k];
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = WB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const int64_t out0 = red[0];
    const int k = knot_of(B, bin_width, n_int);
    const int64_t r0 = row_off[k], n = row_off[k + 1] - r0;
    for (int64_t r = (int64_t)blockIdx.x * WB + threadIdx.x; r < n; r += (int64_t)gridDim.x * WB) {
        for (int c = 0; c < nc; ++c) data_out[(out0 + r) * nc + c] = data[(r0 + r) * nc + c];
        for (int c = 0; c < nmc; ++c) model_out[(out0 + r) * nmc + c] = model[(r0 + r) * nmc + c];
        if (flags_out) flags_out[out0 + r] = flags ? flags[r0 + r] : (uint8_t)0;
    }
}

// gains[k][p] from the knot values y[p][B] (real) / y[p][n_bins + B] (imaginary):
// amplitude and phase linear between the knots around k, constant beyond the outer knots.
__global__ void bins_to_gains_kernel(int n_int, int n_ant, int n_bins, int bin_width, const float* __restrict__ y,
                                     float2* __restrict__ gains) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_int * n_ant) return;
    const int k = (int)(i / n_ant), p = (int)(i % n_ant);
    const float* yr = y + (int64_t)p * 2 * n_bins;
    const float* yi = yr + n_bins;
    int B = min(k / bin_width, n_bins - 1);
    if (k < knot_of(B, bin_width, n_int)) --B;      // bracket [knot(B), knot(B + 1))
    float2 g;
    if (B < 0) {
        g = make_float2(yr[0], yi[0]);
    } else if (B >= n_bins - 1) {
        g = make_float2(yr[n_bins - 1], yi[n_bins - 1]);
    } else {
        const double ar = yr[B], ai = yi[B], br = yr[B + 1], bi = yi[B + 1];
        const int k0 = knot_of(B, bin_width, n_int), k1 = knot_of(B + 1, bin_width, n_int);
        const double w = (double)(k - k0) / (double)(k1 - k0);
        const double amp = (1.0 - w) * sqrt(ar * ar + ai * ai) + w * sqrt(br * br + bi * bi);
        // phase step: principal argument of z_{B+1} conj(z_B)
        const double step = atan2(bi * ar - br * ai, br * ar + bi * ai);
        const double ph = atan2(ai, ar) + w * step;
        double sn, cs;
        sincos(ph, &sn, &cs);
        g = make_float2((float)(amp * cs), (float)(amp * sn));
    }
    gains[i] = g;
}

// y[p][B] / y[p][n_bins + B] = mean over intervals k within halfwidth of knot B (clipped to
// [0, n_int)) of g_pk conj(g_0k) / |g_0k|, from gains [n_int][1][n_ant][1]
__global__ void gains_to_bins_kernel(int n_int, int n_ant, int n_bins, int bin_width, int halfwidth,
                                     const float2* __restrict__ gains, float* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_ant * n_bins) return;
    const int p = (int)(i / n_bins), B = (int)(i % n_bins);
    const int kn = knot_of(B, bin_width, n_int);
    const int k0 = max(kn - halfwidth, 0), k1 = min(kn + halfwidth + 1, n_int);
    double sr = 0.0, si = 0.0;
    for (int k = k0; k < k1; ++k) {
        const float2 g = gains[(int64_t)k * n_ant + p], g0 = gains[(int64_t)k * n_ant];
        const double a0 = sqrt((double)g0.x * g0.x + (double)g0.y * g0.y);
        const double rr = a0 > 0.0 ? g0.x / a0 : 1.0, ri = a0 > 0.0 ? -g0.y / a0 : 0.0;
        sr += g.x * rr - g.y * ri;
        si += g.x * ri + g.y * rr;
    }
    const double n = (double)(k1 - k0);
    y[(int64_t)p * 2 * n_bins + B] = (float)(sr / n);
    y[(int64_t)p * 2 * n_bins + n_bins + B] = (float)(si / n);
}

__global__ void reset_unconverged_kernel(int n_int, int per_int, int nc, const uint32_t* status, float2* gains) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_int * per_int) return;
    const int k = (int)(i / per_int);
    if (status[k] & WCAL_CONVERGED) return;
    const int c = (int)(i % nc);
    gains[i] = (nc == 1 || c == 0 || c == 3) ? make_float2(1.f, 0.f) : make_float2(0.f, 0.f);
}

}  // namespace

extern "C" {

int wcal_bin_knots(int32_t n_int, int32_t bin_width, int32_t* knots) {
    if (!knots || n_int < 1 || bin_width < 1) return wcal_error(WCAL_EINVAL, "bad argument");
    const int n_bins = (n_int + bin_width - 1) / bin_width;
    for (int B = 0; B < n_bins; ++B) knots[B] = knot_of(B, bin_width, n_int);
    return WCAL_OK;
}

int wcal_gather_knots(const wcal_plan* plan, int32_t bin_width, const wcal_c64* data, const wcal_c64* model,
                      const uint8_t* flags, wcal_c64* data_out, wcal_c64* model_out, uint8_t* flags_out,
                      void* stream) {
    if (!plan || !data || !model || !data_out || !model_out) return wcal_error(WCAL_EINVAL, "NULL argument");
    if (bin_width < 1) return wcal_error(WCAL_EINVAL, "bin_width must be >= 1");
    const wcal_problem& p = plan->prob;
    if (hipSetDevice(plan->device) != hipSuccess) return wcal_error(WCAL_EHIP, "hipSetDevice failed");
    const int n_bins = (p.n_int + bin_width - 1) / bin_width;
    if (n_bins > 65535) return wcal_error(WCAL_ESHAPE, "more than 65535 bins");
    const int64_t max_rows = (int64_t)plan->max_ns * p.n_bl;
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_rows + WB - 1) / WB, 512));
    hipLaunchKernelGGL(gather_knots_kernel, dim3(gx, (unsigned)n_bins), dim3(WB), 0,
                       reinterpret_cast<hipStream_t>(stream), p.n_int, bin_width, plan->d_row_off, p.n_corr,
                       p.n_dir * p.n_corr, reinterpret_cast<const float2*>(data),
                       reinterpret_cast<const float2*>(model), flags, reinterpret_cast<float2*>(data_out),
                       reinterpret_cast<float2*>(model_out), flags_out);
    return hipGetLastError() == hipSuccess ? WCAL_OK : wcal_error(WCAL_EHIP, "launch failed");
}

int wcal_bins_to_gains(int32_t n_int, int32_t n_ant, int32_t bin_width, const float* y, wcal_c64* gains,
                       void* stream) {
    if (!y || !gains || n_int < 1 || n_ant < 1 || bin_width < 1) return wcal_error(WCAL_EINVAL, "bad argument");
    const int n_bins = (n_int + bin_width - 1) / bin_width;
    const int64_t n = (int64_t)n_int * n_ant;
    hipLaunchKernelGGL(bins_to_gains_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), n_int, n_ant, n_bins, bin_width, y,
                       reinterpret_cast<float2*>(gains));
    return hipGetLastError() == hipSuccess ? WCAL_OK : wcal_error(WCAL_EHIP, "launch failed");
}

int wcal_gains_to_bins(int32_t n_int, int32_t n_ant, int32_t bin_width, int32_t halfwidth, const wcal_c64* gains,
                       float* y, void* stream) {
    if (!y || !gains || n_int < 1 || n_ant < 1 || bin_width < 1 || halfwidth < 0)
        return wcal_error(WCAL_EINVAL, "bad argument");
    const int n_bins = (n_int + bin_width - 1) / bin_width;
    const int64_t n = (int64_t)n_ant * n_bins;
    hipLaunchKernelGGL(gains_to_bins_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), n_int, n_ant, n_bins, bin_width, halfwidth,
                       reinterpret_cast<const float2*>(gains), y);
    return hipGetLastError() == hipSuccess ? WCAL_OK : wcal_error(WCAL_EHIP, "launch failed");
}

int wcal_reset_unconverged(wcal_plan* plan, const uint32_t* status, wcal_c64* gains, void* stream) {
    if (!plan || !status || !gains) return wcal_error(WCAL_EINVAL, "NULL argument");
    const wcal_problem& p = plan->prob;
    const int per = p.n_dir * p.n_ant * p.n_corr;
    const int64_t n = (int64_t)p.n_int * per;
    hipLaunchKernelGGL(reset_unconverged_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), p.n_int, per, p.n_corr, status,
                       reinterpret_cast<float2*>(gains));
    return hipGetLastError() == hipSuccess ? WCAL_OK : wcal_error(WCAL_EHIP, "launch failed");
}

}  // extern "C"
