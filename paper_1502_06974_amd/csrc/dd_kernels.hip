// Direction-dependent kernels for gfx950: CohJones (per-antenna Nd x Nd blocks of J^H J,
// Sect. 3.2.2) and AllJones (fully diagonal, residual form, Sect. 3.2.3) for scalar gains.
//
// Gram pass (MFMA): for every baseline b of an interval the augmented Gram
//     [M | d | r]^H [M | d | r]   over the interval's samples,
// where the columns are the Nd model visibilities, the data and (accumulate only) the
// residual.  Its blocks are X_b = sum_s conj(m^c) m^e, Z_b = sum_s conj(m^c) d and
// W_b = sum_s conj(m^c) r.  The gains factor out of the sums over samples (as in the
// cross-direction terms of Sect. 3.2.1): with y^e_pq = m^e conj(g^e_q) the diagonal
// blocks of Eq. JHJ:DD:unpol and the vector of Eq. JHR:DD:unpol are
//     H_p[c][e] += g^c_q conj(g^e_q) X_b[c][e],   c_p[c] += g^c_q Z_b[c]          (row pq)
//     H_q[c][e] += g^c_p conj(g^e_p) conj(X_b[c][e]), c_q[c] += g^c_p conj(Z_b[c]) (row qp)
// One wavefront owns one baseline; each v_mfma_f32_16x16x4f32 consumes 4 samples, with
// lane l holding column l % 16 of sample l / 16.  The complex Gram is formed in a real
// embedding with three MFMAs per 4 samples: Re = Ar^T Ar + Ai^T Ai, T = Ar^T Ai,
// Im = T - T^T.  Flagged samples enter as zeros (selected, not multiplied).
//
// Solve: one workgroup per interval contracts the Gram blocks with the current gains in
// FP64, factors every H_p by Cholesky in FP64 (pivot <= EPS * H_jj = singular, gain
// kept), forms the GN value (CohJones: H_p^-1 c_p; AllJones: g + diag(H_p)^-1 J^H r),
// applies the schedule and the FP64 relative-change test.  In STATS mode the Gram pass
// runs once and one launch iterates every interval; in PASS mode the Gram pass is
// repeated before every update.  A tiled residual pass ends the solve.
#include <cstdlib>

#include "dd_common.h"

using namespace wcal_dev;

namespace {

constexpr int NDMAX = 14;        // Nd + 2 augmented columns fit one 16-wide MFMA tile

// floats per baseline record: X (upper, complex), Z, W (complex), sum |d|^2, count
__host__ __device__ inline int rec_floats(int nd) {
    const int n = 2 * ntri(nd) + 4 * nd + 2;
    return (n + 3) / 4 * 4;
}
__host__ __device__ inline int rec_z(int nd) { return 2 * ntri(nd); }
__host__ __device__ inline int rec_w(int nd) { return 2 * ntri(nd) + 2 * nd; }
__host__ __device__ inline int rec_d2(int nd) { return 2 * ntri(nd) + 4 * nd; }
__host__ __device__ inline int rec_cnt(int nd) { return 2 * ntri(nd) + 4 * nd + 1; }

// ------------------------------------------------------------------ Gram pass
// WITH_R: add the residual column (fixed gains), write R and chi^2 per baseline.
template <bool WITH_R>
__global__ void __launch_bounds__(DT) dd_gram_kernel(DdArgs a, DdState st, int only_active) {
    __shared__ float tile[DT / WAVE][2][256];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int nd = a.n_dir, nbl = a.n_bl, na = a.n_ant;
    const int RS = rec_floats(nd);
    const int kk = lane >> 4;      // sample within the 4-sample chunk
    const int col = lane & 15;     // augmented column
    const int64_t ntask = (int64_t)a.n_int * nbl;
    const bool has_flags = a.flags != nullptr;
    for (;;) {
        // Pop one task per wavefront.  The atomic is issued in uniform control flow (every
        // lane, increment 1 from lane 0 only) and the index is made wave-uniform with
        // readfirstlane: a pop guarded by a lane-0 branch inside this loop lets the
        // compiler split the wavefront so that lanes 1..63 re-enter the loop without
        // popping, and they never leave it.
        const int got = atomicAdd(&st.ctr[0], lane == 0 ? 1 : 0);
        const int task = __builtin_amdgcn_readfirstlane(got);
        if (task >= ntask) break;
        const int k = a.order[task / nbl];
        const int b = task % nbl;
        if (only_active && !st.active[k]) continue;
        const int64_t off = a.row_off[k];
        const int ns = a.ns[k];
        const int p = a.ant1[b], q = a.ant2[b];
        float2 wgt = make_float2(0.f, 0.f);
        if (WITH_R && col < nd) {
            const float2* gk = a.gains_in + (int64_t)k * nd * na;
            wgt = cmulc(gk[col * na + p], gk[col * na + q]);   // g^c_p conj(g^c_q)
        }
        floatx4 crr = {0.f, 0.f, 0.f, 0.f}, cri = {0.f, 0.f, 0.f, 0.f};
        int cnt = 0;
        double chi = 0.0;
        constexpr int U = 4;
        for (int s0 = 0; s0 < ns; s0 += 4 * U) {
            float2 val[U];
            bool use[U];
            int64_t rows[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int s = s0 + 4 * u + kk;
                const bool valid = s < ns;
                rows[u] = off + (int64_t)s * nbl + b;
                use[u] = valid && !(has_flags && a.flags[rows[u]] != 0);
                val[u] = make_float2(0.f, 0.f);
                if (use[u]) {
                    if (col < nd) val[u] = a.model[rows[u] * nd + col];
                    else if (col == nd) val[u] = a.data[rows[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float2 v = val[u];
                if constexpr (WITH_R) {
                    // r = d - sum_c g^c_p m^c conj(g^c_q), summed over the 16 lanes of this sample
                    float2 t = col < nd ? cmul(wgt, v) : make_float2(0.f, 0.f);
#pragma unroll
                    for (int o = 1; o < 16; o <<= 1) {
                        t.x += __shfl_xor(t.x, o, 16);
                        t.y += __shfl_xor(t.y, o, 16);
                    }
                    const float dre = __shfl(v.x, nd, 16), dim = __shfl(v.y, nd, 16);
                    const float2 r = use[u] ? make_float2(dre - t.x, dim - t.y) : make_float2(0.f, 0.f);
                    if (col == nd + 1) v = r;
                    if (col == nd && s0 + 4 * u + kk < ns) {
                        if (a.residual) a.residual[rows[u]] = r;
                        chi += (double)nrm(r);
                    }
                }
                if (col == 0 && use[u]) ++cnt;
                crr = __builtin_amdgcn_mfma_f32_16x16x4f32(v.x, v.x, crr, 0, 0, 0);
                crr = __builtin_amdgcn_mfma_f32_16x16x4f32(v.y, v.y, crr, 0, 0, 0);
                cri = __builtin_amdgcn_mfma_f32_16x16x4f32(v.x, v.y, cri, 0, 0, 0);
            }
        }
        // D[i][j] of the 16x16 result sits in lane 16 * (i / 4) + j, register i % 4
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * (lane >> 4) + r;
            tile[w][0][i * 16 + col] = crr[r];
            tile[w][1][i * 16 + col] = cri[r];
        }
        __builtin_amdgcn_wave_barrier();
        float* rec = st.rec + ((int64_t)k * nbl + b) * RS;
        for (int e = lane; e < 256; e += WAVE) {
            const int i = e >> 4, j = e & 15;
            const float re = tile[w][0][i * 16 + j];
            const float im = tile[w][1][i * 16 + j] - tile[w][1][j * 16 + i];
            if (i <= j && j < nd) {
                const int t = tri(i, j, nd);
                rec[2 * t] = re;
                rec[2 * t + 1] = im;
            } else if (i < nd && j == nd) {
                rec[rec_z(nd) + 2 * i] = re;
                rec[rec_z(nd) + 2 * i + 1] = im;
            } else if (WITH_R && i < nd && j == nd + 1) {
                rec[rec_w(nd) + 2 * i] = re;
                rec[rec_w(nd) + 2 * i + 1] = im;
            } else if (i == nd && j == nd) {
                rec[rec_d2(nd)] = re;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // count and chi^2 of the baseline
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            cnt += __shfl_xor(cnt, o, WAVE);
            if constexpr (WITH_R) chi += __shfl_xor(chi, o, WAVE);
        }
        if (lane == 0) {
            reinterpret_cast<int*>(rec)[rec_cnt(nd)] = cnt;
            if constexpr (WITH_R) st.chi_bl[(int64_t)k * nbl + b] = chi;
        }
    }
}

// ------------------------------------------------------------------ Gram passes of the solve
// Work split of the solve's Gram passes: a workgroup owns GB consecutive baselines of one
// interval and walks its samples in chunks; for each sample the model rows of the GB
// baselines are one contiguous segment (GB * Nd complex), so a chunk is read with
// consecutive addresses across the workgroup.  Wavefront w runs the MFMAs of baselines
// 4w .. 4w + 3 (lane l: column l % 16 of sample l / 16, as in the per-baseline kernel above).
constexpr int GB = 16;                 // baselines per workgroup task
typedef short shortx4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest, ties to even (infinities and NaN stay non-finite)
__device__ __forceinline__ short bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(short b) { return __uint_as_float((uint32_t)(uint16_t)b << 16); }

// x from the lane given by a DPP control within the same row of 16 lanes
template <int CTRL>
__device__ __forceinline__ float dpp16(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}
// Sum over each row of 16 lanes, left in every lane of the row: butterfly over the lane
// partners i^1, i^2 (quad permutations), i^7 (half-row mirror) and i^15 (row mirror), whose
// masks span the 16 lanes.  Call with every lane active.
__device__ __forceinline__ float2 row16_sum(float2 v) {
    v.x += dpp16<0xB1>(v.x);  v.y += dpp16<0xB1>(v.y);     // quad_perm [1, 0, 3, 2]
    v.x += dpp16<0x4E>(v.x);  v.y += dpp16<0x4E>(v.y);     // quad_perm [2, 3, 0, 1]
    v.x += dpp16<0x141>(v.x); v.y += dpp16<0x141>(v.y);    // row_half_mirror
    v.x += dpp16<0x140>(v.x); v.y += dpp16<0x140>(v.y);    // row_mirror
    return v;
}

// exp(i x) for an FP64 angle x (|x| < 2^30): the quarter-turn count q (nearest integer to
// x / (pi / 2)) and the remainder r = x - q pi / 2, |r| <= pi / 4, are taken in FP64; sin r
// and cos r are their Taylor series in FP32, through r^9 and r^10 (the first terms left out
// are below 2e-9 on |r| <= pi / 4), turned by q quarter turns.
__device__ __forceinline__ float2 cis_quarter(double x) {
    const double q = rint(x * 0.63661977236758134);
    const float r = (float)fma(-q, 1.5707963267948966, x);
    const float r2 = r * r;
    const float sn = r * fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, 1.f / 362880.f, -1.f / 5040.f), 1.f / 120.f), -1.f / 6.f), 1.f);
    const float cs = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.f / 3628800.f, 1.f / 40320.f), -1.f / 720.f), 1.f / 24.f), -0.5f), 1.f);
    const int qi = (int)q & 3;
    const float u = (qi & 1) ? sn : cs, v = (qi & 1) ? cs : sn;
    return make_float2((qi == 1 || qi == 2) ? -u : u, qi >= 2 ? -v : v);
}

// ------------------------------------------------------------------ predicted-model Gram pass
// Point-source models (Sect. 3.2.1, m^d = S_d exp(-2 pi i (u . sigma_d) nu / c)) generated in
// the MFMA operand layout.  Wavefront w of a task owns PBW consecutive baselines and walks
// their samples four at a time, lane l holding column l % 16 of sample 4g + l / 16 (as in the
// read-model passes).  A lane of model column d keeps one phasor per baseline for its own sample and
// steps it by exp(-2 pi i phi 4 dfreq) from one group to the next; the phasor is re-based
// whenever the lane's sample enters a new time slot and after PREBASE steps, so the walk runs in
// segments between re-bases with a branch-free inner loop.  A re-base reads the phasor and the
// step from the solve's phasor table (dd_phasor_kernel, formed once per solve from the FP64
// phase): a lane enters a slot at a channel below 4 and re-bases every 64 channels, so the
// table holds channels 64 j + r, r < 4, of every (interval, slot, baseline, direction).  Data and flags
// pass through the wavefront's own LDS slice, PCH samples at a time (each lane loads one
// sample of the wavefront's baselines, a chunk ahead): the slice holds the data value, zeroed
// where the row is flagged or absent, and a weight 1 or 0.  Every lane then forms its operand
// as a product, v = z * P: model lanes take P = (weight, weight), the data lane keeps
// z = (1, 1) and takes P = the data value, and lanes past column Nd keep z = 0.  Without
// flags (PLAIN) no row inside the interval has weight 0, so z itself is the operand: the step
// becomes z <- z * step + P, where model lanes read P = 0 (their slice holds zeros) and the
// data lane, whose step is 0, reads the next group's data; only an interval's last group, when
// it is partial, zeroes the z of its absent samples first.  The wavefronts of a task meet only
// at the task pop.
constexpr int PREBASE = 16;
static_assert(PREBASE * 4 == 64, "the phasor table holds one segment per 64 channels");

// The phasor table of a predicted-model solve: one thread per (interval, time slot, baseline,
// direction) forms the FP64 phase phi = -2 pi (u . sigma_d) / c once and writes the step
// exp(i phi 4 dfreq) and, for every 64-channel segment j, S_d exp(i phi nu) at channels 64 j + r,
// r < 4 (zero past the last channel), each exp(i x) by cis_quarter.
__global__ void __launch_bounds__(DT) dd_phasor_kernel(DdArgs a) {
    const int nd = a.n_dir, nch = a.pt.n_chan, nseg = a.pt.nseg;
    const int64_t n = (int64_t)a.n_int * a.pt.n_time * a.n_bl * nd;
    const double sc = -6.283185307179586 / 299792458.0;
    for (int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x; i < n; i += (int64_t)gridDim.x * DT) {
        const int d = (int)(i % nd);
        const int64_t tb = i / nd;   // (k * n_time + t) * n_bl + b
        const double* u = a.pt.uvw + tb * 3;
        const double sg0 = sc * a.pt.lmn[3 * d], sg1 = sc * a.pt.lmn[3 * d + 1], sg2 = sc * a.pt.lmn[3 * d + 2];
        const double ph = u[0] * sg0 + u[1] * sg1 + u[2] * sg2;
        const float flux = a.pt.flux[d];
        a.pt.st[i] = cis_quarter(ph * (4.0 * a.pt.dfreq));
        float2* zo = a.pt.zt + tb * nseg * 4 * nd + d;
        for (int j = 0; j < nseg; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = 64 * j + r;
                float2 z = make_float2(0.f, 0.f);
                if (f < nch) {
                    const float2 e = cis_quarter(ph * (a.pt.freq0 + f * a.pt.dfreq));
                    z = make_float2(flux * e.x, flux * e.y);
                }
                zo[(4 * j + r) * nd] = z;
            }
        }
    }
}
// The FP32 MFMA accumulators of the Gram passes hold the sums of one block of samples; every
// block the sums move into a second set of FP32 accumulators and the MFMA ones start again
// from zero.  A single FP32 chain over a whole interval (1920 samples) loses the gains of faint
// directions: their model-data sums are small against the running sums, which the bright
// sources make large, so their rounding grows with the chain; 128-sample blocks keep it near
// the level of the inputs' own rounding (the chain of at most 128 samples inside a block
// dominates the rounding; FP64 block totals would double the registers for ~30% less error).
constexpr int FOLD_SAMPLES = 128;
template <int NB>
__device__ __forceinline__ void fold_block(floatx4 (&crr)[NB], floatx4 (&cri)[NB], floatx4 (&trr)[NB],
                                           floatx4 (&tri)[NB]) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        trr[j] += crr[j];
        tri[j] += cri[j];
        crr[j] = floatx4{0.f, 0.f, 0.f, 0.f};
        cri[j] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
}

constexpr int PCH = 64;   // samples per staged chunk: one per lane
constexpr int PBW = 4;    // baselines per wavefront
constexpr int PGB = (DT / WAVE) * PBW;   // baselines per task
template <bool PLAIN>
__global__ void __launch_bounds__(DT) __attribute__((amdgpu_waves_per_eu(3, 8))) dd_gram_pts_kernel(DdArgs a, DdState st, const int32_t* list, const int32_t* n_list) {
    // per wavefront: [0] [sample][baseline] data, [1] [sample][baseline] (weight, weight) (PLAIN:
    // zeros), each followed by three groups of padding that the read-ahead after a chunk's last
    // groups lands in (zero: PLAIN's step after a chunk's last group adds it to z); slice 0 also
    // holds the 512-float record tile
    __shared__ float2 sbuf[DT / WAVE][2][(PCH + 12) * PBW];
    __shared__ int s_task;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int nd = a.n_dir, nbl = a.n_bl;
    const int RS = rec_floats(nd);
    const int kk = lane >> 4, col = lane & 15;
    const int nbb = (nbl + PGB - 1) / PGB;
    const int nint = list ? *n_list : a.n_int;
    const int64_t ntask = (int64_t)nint * nbb;
    if ((int64_t)blockIdx.x >= ntask) return;   // tasks are popped dynamically
    const bool has_flags = a.flags != nullptr;
    const bool is_m = col < nd, is_d = col == nd;
    const int nch = a.pt.n_chan, nt = a.pt.n_time, nseg = a.pt.nseg;
    const float2* src = sbuf[w][is_d ? 0 : 1];   // this lane's operand factors
    for (int e = lane; e < (PCH + 12) * PBW; e += WAVE) {
        if (PLAIN || e >= PCH * PBW) sbuf[w][1][e] = make_float2(0.f, 0.f);
        if (e >= PCH * PBW) sbuf[w][0][e] = make_float2(0.f, 0.f);
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_task = atomicAdd(&st.ctr[0], 1);
        __syncthreads();
        const int task = __builtin_amdgcn_readfirstlane(s_task);
        if (task >= ntask) break;
        const int k = list ? list[task / nbb] : a.order[task / nbb];
        const int bw = (task % nbb) * PGB + PBW * w;   // this wavefront's first baseline
        const int nv = min(PBW, nbl - bw);             // its baselines inside the interval (may be <= 0)
        if (nv <= 0) continue;
        const int64_t off = a.row_off[k];
        const int ns = a.ns[k];
        floatx4 crr[PBW], cri[PBW];          // FP32 sums of the current block of samples
        floatx4 trr[PBW], tri4[PBW];         // sums of the finished blocks
        int cnt[PBW];
        float2 z[PBW], stp[PBW];
#pragma unroll
        for (int j = 0; j < PBW; ++j) {
            crr[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            cri[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            trr[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            tri4[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            cnt[j] = 0;
            z[j] = is_d && !PLAIN ? make_float2(1.f, 1.f) : make_float2(0.f, 0.f);
            stp[j] = is_d && !PLAIN ? make_float2(1.f, 0.f) : make_float2(0.f, 0.f);
        }
        // the lane's sample (kk + 4g) sits at time slot t, channel f (f may run past the slot
        // until the next re-base); left counts the groups its phasor stays valid for
        int t = 0, f = kk, left = 0;
        // chunk staging: lane l loads sample c PCH + l of the wavefront's baselines (clamped
        // rows keep every address inside the interval)
        float2 pd[PBW];
        int pf[PBW];
        auto fetch = [&](int c) {
            const int sc = min(c * PCH + lane, ns - 1);
            const int64_t r0 = off + (int64_t)sc * nbl + bw;
#pragma unroll
            for (int j = 0; j < PBW; ++j) {
                const int jc = min(j, nv - 1);
                pd[j] = a.data[r0 + jc];
                pf[j] = has_flags ? (int)a.flags[r0 + jc] : 0;
            }
        };
        const int nchunk = (ns + PCH - 1) / PCH;
        fetch(0);
        for (int c = 0; c < nchunk; ++c) {
            __builtin_amdgcn_wave_barrier();
            {
                const bool sv = c * PCH + lane < ns;
#pragma unroll
                for (int j = 0; j < PBW; ++j) {
                    const bool ok = sv && j < nv && pf[j] == 0;
                    const float wv = ok ? 1.f : 0.f;
                    sbuf[w][0][lane * PBW + j] = ok ? pd[j] : make_float2(0.f, 0.f);
                    if (!PLAIN) sbuf[w][1][lane * PBW + j] = make_float2(wv, wv);
                    cnt[j] += ok ? 1 : 0;
                }
            }
            __builtin_amdgcn_wave_barrier();
            const int ng = min(PCH / 4, (ns - c * PCH + 3) / 4);
            // staged factors, read two groups ahead of their use: operand factors of groups gg (Pa)
            // and gg + 1 (Pb); PLAIN: the step's addends, of groups gg + 1 and gg + 2
            constexpr int O = PLAIN ? 1 : 0;
            float2 Pa[PBW], Pb[PBW];
#pragma unroll
            for (int j = 0; j < PBW; ++j) {
                Pa[j] = src[(4 * O + kk) * PBW + j];
                Pb[j] = src[(4 * O + 4 + kk) * PBW + j];
                if (PLAIN && is_d) z[j] = src[kk * PBW + j];   // the data lane's z: its own data
            }
            int gg = 0;
            while (gg < ng) {
                if (left == 0) {
                    // re-base: the lane's sample enters a new time slot or has taken PREBASE steps
                    while (f >= nch) {
                        f -= nch;
                        ++t;
                    }
                    if (is_m && 4 * (c * (PCH / 4) + gg) + kk < ns) {
                        // phasors of the solve's table: segment f / 64, channel f % 64 < 4
                        const int64_t tb = ((int64_t)k * nt + t) * nbl + bw;
                        const float2* zr = a.pt.zt + ((tb * nseg + (f >> 6)) * 4 + (f & 63)) * nd + col;
                        const float2* sr = a.pt.st + tb * nd + col;
#pragma unroll
                        for (int j = 0; j < PBW; ++j) {
                            if (j < nv) {
                                z[j] = zr[(int64_t)j * nseg * 4 * nd];
                                stp[j] = sr[j * nd];
                            }
                        }
                    }
                    // the phasors have arrived before the chunk read-ahead below is issued:
                    // a wait for them inside the walk would also wait for the read-ahead
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
                    left = min(PREBASE, (nch - f + 3) / 4);
                }
                // groups until the first of the wavefront's four sample rows needs a re-base
                // (lanes of one row, l / 16, share their state)
                int seg = min(__builtin_amdgcn_readlane(left, 0), __builtin_amdgcn_readlane(left, 16));
                seg = min(seg, min(__builtin_amdgcn_readlane(left, 32), __builtin_amdgcn_readlane(left, 48)));
                seg = min(seg, ng - gg);
                if (PLAIN) {
                    // an interval's partial last group runs alone, with the z of its absent samples zeroed
                    const int gf = (ns - c * PCH) / 4;   // groups of the chunk that lie inside the interval
                    if (gg < gf) {
                        seg = min(seg, gf - gg);
                    } else if (4 * (c * (PCH / 4) + gg) + kk >= ns) {
#pragma unroll
                        for (int j = 0; j < PBW; ++j) z[j] = make_float2(0.f, 0.f);
                    }
                }
                if (gg == 0 && c + 1 < nchunk) fetch(c + 1);   // behind the re-base's uvw loads
                // one group: operands from z and the staged factors P, which then take group
                // g + 2's (after a chunk's last groups: the padding), three MFMAs per baseline,
                // step z.  PLAIN: z is the operand, the step adds P (group g + 1's addend), and
                // P then takes group g + 3's
                auto group = [&](int g, float2 (&P)[PBW]) {
                    if constexpr (PLAIN) {
#pragma unroll
                        for (int j = 0; j < PBW; ++j) {
                            crr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(z[j].x, z[j].x, crr[j], 0, 0, 0);
                            crr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(z[j].y, z[j].y, crr[j], 0, 0, 0);
                            cri[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(z[j].x, z[j].y, cri[j], 0, 0, 0);
                        }
#pragma unroll
                        for (int j = 0; j < PBW; ++j) {
                            z[j] = make_float2(fmaf(z[j].x, stp[j].x, fmaf(-z[j].y, stp[j].y, P[j].x)),
                                               fmaf(z[j].x, stp[j].y, fmaf(z[j].y, stp[j].x, P[j].y)));
                        }
                        const float2* pr = src + (4 * g + 12 + kk) * PBW;
#pragma unroll
                        for (int j = 0; j < PBW; ++j) P[j] = pr[j];
                    } else {
                        float vx[PBW], vy[PBW];
#pragma unroll
                        for (int j = 0; j < PBW; ++j) {
                            vx[j] = z[j].x * P[j].x;
                            vy[j] = z[j].y * P[j].y;
                        }
                        const float2* pr = src + (4 * g + 8 + kk) * PBW;
#pragma unroll
                        for (int j = 0; j < PBW; ++j) P[j] = pr[j];
#pragma unroll
                        for (int j = 0; j < PBW; ++j) {
                            crr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(vx[j], vx[j], crr[j], 0, 0, 0);
                            crr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(vy[j], vy[j], crr[j], 0, 0, 0);
                            cri[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(vx[j], vy[j], cri[j], 0, 0, 0);
                        }
#pragma unroll
                        for (int j = 0; j < PBW; ++j) z[j] = cmul(z[j], stp[j]);
                    }
                };
                // two groups per trip (a loop-carried z then needs no register copies); after an
                // odd count the next group's factors are in Pb
                const int ge = gg + seg;
                for (; gg + 1 < ge; gg += 2) {
                    group(gg, Pa);
                    group(gg + 1, Pb);
                }
                if (gg < ge) {
                    group(gg++, Pa);
#pragma unroll
                    for (int j = 0; j < PBW; ++j) {
                        const float2 t = Pa[j];
                        Pa[j] = Pb[j];
                        Pb[j] = t;
                    }
                }
                left -= seg;
                f += 4 * seg;
            }
            if ((c + 1) % (FOLD_SAMPLES / PCH) == 0 || c + 1 == nchunk) fold_block<PBW>(crr, cri, trr, tri4);
        }
        // records of the wavefront's baselines, through its own LDS slice
        __builtin_amdgcn_wave_barrier();
        float* tile = reinterpret_cast<float*>(&sbuf[w][0][0]);
#pragma unroll
        for (int j = 0; j < PBW; ++j) {
            const int b = bw + j;
            int cj = cnt[j];
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) cj += __shfl_xor(cj, o, WAVE);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * kk + r;
                tile[i * 16 + col] = trr[j][r];
                tile[256 + i * 16 + col] = tri4[j][r];
            }
            __builtin_amdgcn_wave_barrier();
            if (b < nbl) {
                float* rec = st.rec + ((int64_t)k * nbl + b) * RS;
                for (int e = lane; e < 256; e += WAVE) {
                    const int i = e >> 4, jj = e & 15;
                    const float re = tile[i * 16 + jj];
                    const float im = tile[256 + i * 16 + jj] - tile[256 + jj * 16 + i];
                    if (i <= jj && jj < nd) {
                        const int tt = tri(i, jj, nd);
                        rec[2 * tt] = re;
                        rec[2 * tt + 1] = im;
                    } else if (i < nd && jj == nd) {
                        rec[rec_z(nd) + 2 * i] = re;
                        rec[rec_z(nd) + 2 * i + 1] = im;
                    } else if (i == nd && jj == nd) {
                        rec[rec_d2(nd)] = re;
                    }
                }
                if (lane == 0) reinterpret_cast<int*>(rec)[rec_cnt(nd)] = cj;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// BF16 Gram pass (plan precision WCAL_PREC_BF16_GRAM): the products are taken by
// v_mfma_f32_16x16x16_bf16, 16 samples per MFMA (lane l holds 4 consecutive samples of
// column l % 16, starting at sample 4 (l / 16)), from values rounded to BF16 (nearest, ties
// to even), accumulated in FP32.  With the MFMA work this small the pass is a stream: the
// model rows are copied straight from HBM into LDS (global_load_lds), with no register
// staging, so more workgroups fit per CU and hide each other's copy phases.  Same work split
// and copy as dd_gram_dmaf_kernel, chunks of GSD = 16 samples.  The model rows of a chunk land in LDS
// in their HBM order, [sample][baseline][Nd], as pieces of PIECE bytes: 16 when Nd is even
// and the model array is 16-byte aligned (every sample's segment is then 16-byte aligned),
// else 4.  Data and flags (9 B per row) go through registers.  Columns Nd + 1 and Nd + 2
// carry the residual r = d - sum_c g^c_p m^c conj(g^c_q), formed in FP32 from the current
// gains and split into its BF16 rounding and the remainder (so M^H r keeps ~16 bits of r),
// and the update takes the residual form g + H^-1 J^H r: its fixed point is that of the
// exact sums up to the fixed rounding of M, although H comes from BF16 products.  A single
// BF16 column for r would make J^H r jump with the rounding of r as the gains move, and
// the iteration would chatter above the tolerance instead of converging.  Needs Nd <= 13.
// (A double-buffered copy serialises: the compiler waits for every outstanding copy before
// any LDS read.)  Five waves per SIMD (94 VGPRs, no spills; the static LDS allows no more):
// 32.2 -> 29.0 ms of pass per cohjones_na64 solve against four.
constexpr int GSD = 16;

template <int PIECE>
__global__ void __launch_bounds__(DT) __attribute__((amdgpu_waves_per_eu(5))) dd_gram_dma_kernel(DdArgs a, DdState st, const int32_t* list, const int32_t* n_list) {
    __shared__ __align__(16) float2 mbuf[GSD * GB * NDMAX];
    __shared__ float2 dbuf[GSD][GB];
    __shared__ uint8_t fbuf[GSD][GB];
    __shared__ int s_task;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int nd = a.n_dir, nbl = a.n_bl;
    const int RS = rec_floats(nd);
    const int kk = lane >> 4;
    const int col = lane & 15;
    const int nbb = (nbl + GB - 1) / GB;
    const int nint = list ? *n_list : a.n_int;
    const int64_t ntask = (int64_t)nint * nbb;
    if ((int64_t)blockIdx.x >= ntask) return;   // tasks are popped dynamically
    const bool has_flags = a.flags != nullptr;
    const int seg_bytes = GB * nd * 8;          // one sample's model segment
    const int npass = (seg_bytes / PIECE + WAVE - 1) / WAVE;   // copies of 64 pieces per segment
    const int ds = threadIdx.x / GB, db = threadIdx.x % GB;   // data / flag element of this thread
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_task = atomicAdd(&st.ctr[0], 1);
        __syncthreads();
        const int task = __builtin_amdgcn_readfirstlane(s_task);
        if (task >= ntask) break;
        const int k = list ? list[task / nbb] : a.order[task / nbb];
        const int b0 = (task % nbb) * GB;
        const int64_t off = a.row_off[k];
        const int ns = a.ns[k];
        const int nch = (ns + GSD - 1) / GSD;
        const int seg_have = min(GB, nbl - b0) * nd * 8;   // bytes of a segment that exist
        floatx4 crr[4], cri[4];
        int cnt[4];
        float2 wgt[4];           // g^c_p conj(g^c_q) of this lane's column for its 4 baselines
        const float2* gk = a.gains + (int64_t)k * nd * a.n_ant;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            crr[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            cri[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            cnt[j] = 0;
            const int b = b0 + 4 * w + j;
            wgt[j] = make_float2(0.f, 0.f);
            if (b < nbl && col < nd) wgt[j] = cmulc(gk[col * a.n_ant + a.ant1[b]], gk[col * a.n_ant + a.ant2[b]]);
        }
        for (int c = 0; c < nch; ++c) {
            const int s0 = c * GSD;
            // model: each wavefront copies the segments of samples w, w + 4, ... of the chunk,
            // 64 pieces at a time, from a uniform base (as dd_gram_dmaf_kernel)
            for (int sm = w; sm < GSD && s0 + sm < ns; sm += DT / WAVE) {
                const char* seg = reinterpret_cast<const char*>(a.model + (off + (int64_t)(s0 + sm) * nbl + b0) * nd);
                char* lds = reinterpret_cast<char*>(mbuf) + sm * seg_bytes;
                for (int h = 0; h < npass; ++h) {
                    const int jb = (h * WAVE + lane) * PIECE;
                    if (jb < seg_have) {
                        auto dst = (__attribute__((address_space(3))) void*)(lds + h * WAVE * PIECE);
                        if constexpr (PIECE == 16) __builtin_amdgcn_global_load_lds(seg + jb, dst, 16, 0, 0);
                        else __builtin_amdgcn_global_load_lds(seg + jb, dst, 4, 0, 0);
                    }
                }
            }
            {
                const bool ok = s0 + ds < ns && b0 + db < nbl;
                const int64_t row = off + (int64_t)(s0 + ds) * nbl + b0 + db;
                dbuf[ds][db] = ok ? a.data[row] : make_float2(0.f, 0.f);
                fbuf[ds][db] = ok ? (has_flags ? (uint8_t)(a.flags[row] != 0) : (uint8_t)0) : (uint8_t)1;
            }
            __syncthreads();     // the model pieces have landed (the barrier waits for them)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int bl = 4 * w + j;
                shortx4 re, im;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int sl = 4 * kk + i;
                    const bool use = !fbuf[sl][bl];
                    float2 v = make_float2(0.f, 0.f);
                    if (use && col < nd) v = mbuf[(sl * GB + bl) * nd + col];
                    else if (use && col == nd) v = dbuf[sl][bl];
                    if (use && col == 0) ++cnt[j];
                    // residual r = d - sum_c g^c_p m^c conj(g^c_q) in FP32: lane col < nd holds
                    // -g m conj(g) of its direction, lane nd holds d, and one butterfly over
                    // the 16 lanes of the sample leaves r in each of them
                    float2 t = col == nd ? v : cmul(wgt[j], v);
                    if (col < nd) { t.x = -t.x; t.y = -t.y; }
                    t = row16_sum(t);
                    const float2 r = use ? t : make_float2(0.f, 0.f);
                    // r in two BF16 columns: nd + 1 the rounded value, nd + 2 what rounding left
                    if (col == nd + 1) v = r;
                    if (col == nd + 2)
                        v = make_float2(r.x - bf16_value(bf16_bits(r.x)), r.y - bf16_value(bf16_bits(r.y)));
                    re[i] = bf16_bits(v.x);
                    im[i] = bf16_bits(v.y);
                }
                crr[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(re, re, crr[j], 0, 0, 0);
                crr[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(im, im, crr[j], 0, 0, 0);
                cri[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(re, im, cri[j], 0, 0, 0);
            }
            __syncthreads();     // every wavefront is done with this chunk before the next lands
        }
        // epilogue through each wavefront's own 2 x 256 floats of mbuf (free now)
        float* tile = reinterpret_cast<float*>(mbuf) + w * 512;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + 4 * w + j;
            int cj = cnt[j];
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) cj += __shfl_xor(cj, o, WAVE);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * (lane >> 4) + r;
                tile[i * 16 + col] = crr[j][r];
                tile[256 + i * 16 + col] = cri[j][r];
            }
            __builtin_amdgcn_wave_barrier();
            if (b < nbl) {
                float* rec = st.rec + ((int64_t)k * nbl + b) * RS;
                for (int e = lane; e < 256; e += WAVE) {
                    const int i = e >> 4, jj = e & 15;
                    const float re = tile[i * 16 + jj];
                    const float im = tile[256 + i * 16 + jj] - tile[256 + jj * 16 + i];
                    if (i <= jj && jj < nd) {
                        const int t = tri(i, jj, nd);
                        rec[2 * t] = re;
                        rec[2 * t + 1] = im;
                    } else if (i < nd && jj == nd) {
                        rec[rec_z(nd) + 2 * i] = re;
                        rec[rec_z(nd) + 2 * i + 1] = im;
                    } else if (i < nd && jj == nd + 1) {
                        // J^H r from the two residual columns
                        rec[rec_w(nd) + 2 * i] = re + tile[i * 16 + jj + 1];
                        rec[rec_w(nd) + 2 * i + 1] = im + tile[256 + i * 16 + jj + 1] - tile[256 + (jj + 1) * 16 + i];
                    } else if (i == nd && jj == nd) {
                        rec[rec_d2(nd)] = re;
                    }
                }
                if (lane == 0) reinterpret_cast<int*>(rec)[rec_cnt(nd)] = cj;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

constexpr int GSF = 16;   // samples per chunk of dd_gram_dmaf_kernel
typedef float lds_f2 __attribute__((ext_vector_type(2)));   // an operand read from LDS
constexpr int GFOLD = FOLD_SAMPLES / GSF;   // chunks per FP64 fold
// dynamic LDS of dd_gram_dmaf_kernel: a chunk's model rows, at least the 4 x 512-float
// epilogue tiles
inline size_t dmaf_smem_bytes(int nd) {
    const size_t n = (size_t)GSF * GB * nd;
    return (n > 1024 ? n : 1024) * sizeof(float2);
}


// The FP32 Gram pass of the solve (no residual column): the model rows of a chunk of GSF
// samples are copied straight from HBM into LDS (global_load_lds, no register staging, so
// the copy costs no vector instructions, which on this part do not overlap the MFMAs).  Data and
// flags go through registers; a chunk that holds a flagged or absent row (a block-wide OR at
// the barrier) gets those rows' model values zeroed in LDS before use (a selection, so
// non-finite values under a flag never reach a product).  Each lane reads its operand with
// one base and stride: model column col < Nd, the data column Nd, or a zero slot.
// Vector instructions do not issue beside the MFMAs, so the pass is bound by the issue of
// both, and resident wavefronts hide the chunk's memory round trip: five per SIMD (95 VGPRs,
// no spills) against three at the compiler's own choice, 26.1 -> 22.9 ms of pass per
// cohjones_na64 solve (four: 24.5 ms; six spill and run 26.8 ms).
template <int PIECE>
__global__ void __launch_bounds__(DT) __attribute__((amdgpu_waves_per_eu(5))) dd_gram_dmaf_kernel(DdArgs a, DdState st, const int32_t* list, const int32_t* n_list) {
    extern __shared__ __align__(16) float2 mbuf[];   // dmaf_smem_bytes(Nd)
    __shared__ float2 dbuf[GSF * GB + 1];      // the last slot stays zero
    __shared__ int s_cnt[GB];
    __shared__ int s_task;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int nd = a.n_dir, nbl = a.n_bl;
    const int RS = rec_floats(nd);
    const int kk = lane >> 4;
    const int col = lane & 15;
    const int nbb = (nbl + GB - 1) / GB;
    const int nint = list ? *n_list : a.n_int;
    const int64_t ntask = (int64_t)nint * nbb;
    if ((int64_t)blockIdx.x >= ntask) return;   // tasks are popped dynamically
    const bool has_flags = a.flags != nullptr;
    const int seg_bytes = GB * nd * 8;          // one sample's model segment
    const int npass = (seg_bytes / PIECE + WAVE - 1) / WAVE;   // copies of 64 pieces per segment
    // this lane's operand: element (sample sl, baseline bl) at base[(sl GB + bl) * stride]
    const float2* obase = col < nd ? mbuf + col : col == nd ? dbuf : dbuf + GSF * GB;
    const int ostride = col < nd ? nd : col == nd ? 1 : 0;
    // the lane's operand (sample 4 g + kk, baseline 4 w + j) sits at LDS byte ob0 + g sg + j sj
    const uint32_t ob0 = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float2*)(obase + (kk * GB + 4 * w) * ostride);
    const uint32_t sj = (uint32_t)ostride * 8u, sg = 4u * GB * (uint32_t)ostride * 8u;
    // this thread's row of every chunk: sample si, baseline bi
    static_assert(GSF * GB == DT, "one staged row per thread");
    const int si = threadIdx.x / GB, bi = threadIdx.x % GB;
    if (threadIdx.x == 0) dbuf[GSF * GB] = make_float2(0.f, 0.f);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_task = atomicAdd(&st.ctr[0], 1);
        if (threadIdx.x < GB) s_cnt[threadIdx.x] = 0;
        __syncthreads();
        const int task = __builtin_amdgcn_readfirstlane(s_task);
        if (task >= ntask) break;
        const int k = list ? list[task / nbb] : a.order[task / nbb];
        const int b0 = (task % nbb) * GB;
        const int64_t off = a.row_off[k];
        const int ns = a.ns[k];
        const int nch = (ns + GSF - 1) / GSF;
        const int seg_have = min(GB, nbl - b0) * nd * 8;   // bytes of a segment that exist
        const bool bi_ok = b0 + bi < nbl;
        int cnt = 0;                                       // unflagged rows of this thread
        floatx4 crr[4], cri[4];   // sums of the current block of GFOLD chunks
        floatx4 trr[4], tri4[4];  // sums of the finished blocks
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            crr[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            cri[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            trr[j] = floatx4{0.f, 0.f, 0.f, 0.f};
            tri4[j] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        for (int cb = 0; cb < nch; cb += GFOLD) {
        const int ce = min(nch, cb + GFOLD);
        for (int c = cb; c < ce; ++c) {
            const int s0 = c * GSF;
            // model: each wavefront copies the segments of samples w, w + 4, ... of the chunk,
            // 64 pieces at a time (lane l: piece h 64 + l); the segment's base is uniform, so
            // the address arithmetic stays scalar
            for (int sm = w; sm < GSF && s0 + sm < ns; sm += DT / WAVE) {
                const char* seg = reinterpret_cast<const char*>(a.model + (off + (int64_t)(s0 + sm) * nbl + b0) * nd);
                char* lds = reinterpret_cast<char*>(mbuf) + sm * seg_bytes;
                for (int h = 0; h < npass; ++h) {
                    const int jb = (h * WAVE + lane) * PIECE;
                    if (jb < seg_have) {
                        auto dst = (__attribute__((address_space(3))) void*)(lds + h * WAVE * PIECE);
                        if constexpr (PIECE == 16) __builtin_amdgcn_global_load_lds(seg + jb, dst, 16, 0, 0);
                        else __builtin_amdgcn_global_load_lds(seg + jb, dst, 4, 0, 0);
                    }
                }
            }
            // data and flag of this thread's row, both requested before either is used (the
            // data of a flagged row is read and dropped by a selection)
            const bool ok = s0 + si < ns && bi_ok;
            const int64_t row = off + (int64_t)(s0 + si) * nbl + b0 + bi;
            float2 dv = make_float2(0.f, 0.f);
            uint8_t fl = 0;
            if (ok) {
                dv = a.data[row];
                if (has_flags) fl = a.flags[row];
            }
            const bool sk = !ok || fl != 0;
            dbuf[threadIdx.x] = sk ? make_float2(0.f, 0.f) : dv;
            cnt += sk ? 0 : 1;
            // the model pieces have landed (the barrier waits for them); a flagged or absent
            // row is cleared by its own thread
            if (__syncthreads_or(sk)) {
                if (sk) {
                    float2* mr = mbuf + threadIdx.x * nd;
                    for (int e = 0; e < nd; ++e) mr[e] = make_float2(0.f, 0.f);
                }
                __syncthreads();
            }
            // the operand addresses are formed again for every chunk from an opaque base, so
            // that 16 of them do not stay live (in registers) across the chunk loop
            uint32_t ob = ob0;
            asm volatile("" : "+v"(ob));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
#pragma unroll
                for (int g = 0; g < GSF / 4; ++g) {
                    const lds_f2 v = *(const __attribute__((address_space(3))) lds_f2*)(uintptr_t)(ob + g * sg + j * sj);
                    crr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(v.x, v.x, crr[j], 0, 0, 0);
                    crr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(v.y, v.y, crr[j], 0, 0, 0);
                    cri[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(v.x, v.y, cri[j], 0, 0, 0);
                }
            }
            __syncthreads();     // every wavefront is done with this chunk before the next lands
        }
        fold_block<4>(crr, cri, trr, tri4);
        }
        atomicAdd(&s_cnt[bi], cnt);
        __syncthreads();
        // epilogue through each wavefront's own 2 x 256 floats of mbuf (free now)
        float* tile = reinterpret_cast<float*>(mbuf) + w * 512;
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + 4 * w + j;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * (lane >> 4) + r;
                tile[i * 16 + col] = trr[j][r];
                tile[256 + i * 16 + col] = tri4[j][r];
            }
            __builtin_amdgcn_wave_barrier();
            if (b < nbl) {
                float* rec = st.rec + ((int64_t)k * nbl + b) * RS;
                for (int e = lane; e < 256; e += WAVE) {
                    const int i = e >> 4, jj = e & 15;
                    const float re = tile[i * 16 + jj];
                    const float im = tile[256 + i * 16 + jj] - tile[256 + jj * 16 + i];
                    if (i <= jj && jj < nd) {
                        const int t = tri(i, jj, nd);
                        rec[2 * t] = re;
                        rec[2 * t + 1] = im;
                    } else if (i < nd && jj == nd) {
                        rec[rec_z(nd) + 2 * i] = re;
                        rec[rec_z(nd) + 2 * i + 1] = im;
                    } else if (i == nd && jj == nd) {
                        rec[rec_d2(nd)] = re;
                    }
                }
                if (lane == 0) reinterpret_cast<int*>(rec)[rec_cnt(nd)] = s_cnt[4 * w + j];
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// ------------------------------------------------------------------ per-antenna blocks
constexpr int BA = 16;   // antennas per batch of the per-antenna solve

// For antennas p0 .. p0 + nb - 1 of interval k: H[j][tri] (FP64, upper packed) and C[j][c]
// from the Gram records and the gains G[c][ant] (LDS); WITH_R also J^H r and row counts.
template <bool WITH_R>
__device__ void dd_blocks(const DdArgs& a, const DdState& st, int k, const float2* G, int p0, int nb,
                          double2* H, double2* C, double2* JR, int* CNT) {
    const int nd = a.n_dir, na = a.n_ant, nbl = a.n_bl;
    const int nx = ntri(nd);
    const int per = nx + nd;
    const int RS = rec_floats(nd);
    const float* recs = st.rec + (int64_t)k * nbl * RS;
    for (int task = threadIdx.x; task < nb * per; task += blockDim.x) {
        const int j = task / per, e = task % per;
        const int p = p0 + j;
        int ci = 0, cj = 0;
        if (e < nx) {
            // invert tri(): row ci holds nd - ci entries
            int rem = e;
            while (rem >= nd - ci) { rem -= nd - ci; ++ci; }
            cj = ci + rem;
        } else {
            ci = e - nx;
        }
        double2 acc = make_double2(0.0, 0.0), accr = make_double2(0.0, 0.0);
        int cnt = 0;
        for (int t = st.ant_ptr[p]; t < st.ant_ptr[p + 1]; ++t) {
            const int code = st.ant_bl[t];
            const int b = code >> 1, side = code & 1;
            const int o = side ? a.ant1[b] : a.ant2[b];     // the other antenna of the row
            const float* rec = recs + (int64_t)b * RS;
            const float2 goc = G[ci * na + o];
            if (e < nx) {
                const float2 goe = G[cj * na + o];
                const double2 x = make_double2(rec[2 * e], side ? -rec[2 * e + 1] : rec[2 * e + 1]);
                const double2 wv = make_double2((double)goc.x * goe.x + (double)goc.y * goe.y,
                                                (double)goc.y * goe.x - (double)goc.x * goe.y);   // g^ci conj(g^cj)
                const double2 prod = dmul(wv, x);
                acc.x += prod.x; acc.y += prod.y;
            } else {
                const float* z = rec + rec_z(nd) + 2 * ci;
                const double2 zz = make_double2(z[0], side ? -z[1] : z[1]);
                const double2 prod = dmul(make_double2(goc.x, goc.y), zz);
                acc.x += prod.x; acc.y += prod.y;
                if constexpr (WITH_R) {
                    const float* wr = rec + rec_w(nd) + 2 * ci;
                    const double2 ww = make_double2(wr[0], side ? -wr[1] : wr[1]);
                    const double2 pr = dmul(make_double2(goc.x, goc.y), ww);
                    accr.x += pr.x; accr.y += pr.y;
                    if (ci == 0) cnt += reinterpret_cast<const int*>(rec)[rec_cnt(nd)];
                }
            }
        }
        if (e < nx) H[j * nx + e] = acc;
        else {
            C[j * nd + ci] = acc;
            if constexpr (WITH_R) {
                JR[j * nd + ci] = accr;
                if (ci == 0) CNT[j] = cnt;
            }
        }
    }
}

// H[i][j] of one antenna's packed upper triangle (any i, j)
__device__ __forceinline__ double2 hget(const double2* h, int i, int j, int nd) {
    if (i <= j) return h[tri(i, j, nd)];
    const double2 v = h[tri(j, i, nd)];
    return make_double2(v.x, -v.y);
}

// Forward and back substitution with the Cholesky factor R of H = R^H R (upper, packed,
// as dd_ant_kernel leaves it): R^H z = c, then R x = z.
__device__ void chol_subst(const double2* h, const double2* c, double2* x, int nd) {
    // forward: R^H z = c
    for (int i = 0; i < nd; ++i) {
        double2 v = c[i];
        for (int k = 0; k < i; ++k) {
            const double2 rki = h[tri(k, i, nd)];
            const double2 zk = x[k];
            v.x -= rki.x * zk.x + rki.y * zk.y;     // conj(R[k][i]) z[k]
            v.y -= rki.x * zk.y - rki.y * zk.x;
        }
        const double rii = h[tri(i, i, nd)].x;
        x[i] = make_double2(v.x / rii, v.y / rii);
    }
    // back: R x = z
    for (int i = nd - 1; i >= 0; --i) {
        double2 v = x[i];
        for (int k = i + 1; k < nd; ++k) {
            const double2 p = dmul(h[tri(i, k, nd)], x[k]);
            v.x -= p.x; v.y -= p.y;
        }
        const double rii = h[tri(i, i, nd)].x;
        x[i] = make_double2(v.x / rii, v.y / rii);
    }
}

struct DdSmem {
    double2* H;    // [BA][ntri]
    double2* C;    // [BA][nd]
    double2* X;    // [BA][NDMAX]
    double2* JR;   // [BA][nd]
    int* CNT;      // [BA]
    float2* G;     // [nd][na]
    float2* Gn;    // [nd][na]
};

__host__ __device__ inline size_t dd_smem_size(int nd, int na) {
    return (size_t)BA * (ntri(nd) + 2 * nd + NDMAX) * 16 + (size_t)BA * 4 + 2 * (size_t)nd * na * 8;
}

__device__ DdSmem dd_smem(unsigned char* smem, int nd, int na) {
    DdSmem s;
    s.H = reinterpret_cast<double2*>(smem);
    s.C = s.H + BA * ntri(nd);
    s.X = s.C + BA * nd;
    s.JR = s.X + BA * NDMAX;
    s.CNT = reinterpret_cast<int*>(s.JR + BA * nd);
    s.G = reinterpret_cast<float2*>(s.CNT + BA);
    s.Gn = s.G + nd * na;
    return s;
}


// LDS bytes of the gains [nd][na] in dd_ant_kernel, rounded up to 16 for the FP64 blocks
__host__ __device__ inline size_t ant_g_bytes(int nd, int na) { return ((size_t)nd * na * 8 + 15) / 16 * 16; }
// dynamic LDS of dd_ant_kernel: the gains, then 16-byte slots for the wavefront partials,
// H, c and the solve
inline size_t ant_smem(int nd, int na) {
    return ant_g_bytes(nd, na) + ((size_t)(DT / WAVE) * 2 * WAVE + ntri(nd) + nd + NDMAX) * 16;
}

// One update, per antenna: one workgroup forms H_p and c_p of one antenna.  Lanes run over
// the Nd(Nd+1)/2 + Nd entries; the four wavefronts take every fourth of the antenna's
// baselines (in CSR order, 8 records in flight per lane) and their FP64 sums are folded in
// wavefront order.  CohJones factors H_p across the workgroup (Cholesky); then one lane
// substitutes (CohJones) or takes the diagonal residual-form steps (AllJones), applies the
// schedule and writes the candidate gains and its share of the FP64 relative-change norms.
// The interval's decision follows in dd_finish_kernel.
__global__ void __launch_bounds__(DT) dd_ant_kernel(DdArgs a, DdState st, int it) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nd = a.n_dir, na = a.n_ant, nbl = a.n_bl;
    const int nx = ntri(nd), per = nx + nd;
    const int nw = DT / WAVE;
    const int k = blockIdx.x / na;
    if (!st.active[k]) return;
    const bool resid = a.precision == WCAL_PREC_BF16_GRAM;   // J^H r in C, residual-form update
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int p = blockIdx.x % na;
    float2* G = reinterpret_cast<float2*>(smem);                              // [nd][na]
    double2* part = reinterpret_cast<double2*>(smem + ant_g_bytes(nd, na));   // [nw][2 WAVE]
    double2* H = part + nw * 2 * WAVE;                                         // [nx] then C [nd], X [NDMAX]
    double2* C = H + nx;
    double2* X = C + nd;
    const float2* gk = a.gains + (int64_t)k * nd * na;
    for (int i = threadIdx.x; i < nd * na; i += blockDim.x) G[i] = gk[i];
    __syncthreads();
    {
        const int RS = rec_floats(nd);
        const float* recs = st.rec + (int64_t)k * nbl * RS;
        const int t0 = st.ant_ptr[p], t1 = st.ant_ptr[p + 1];
        for (int e = lane; e < per; e += WAVE) {
            int ci = 0, cj = 0;
            if (e < nx) {
                int rem = e;
                while (rem >= nd - ci) { rem -= nd - ci; ++ci; }
                cj = ci + rem;
            } else {
                ci = e - nx;
            }
            double2 acc = make_double2(0.0, 0.0);
            // the record entry this lane sums: X[e] (block) or, for c_p, Z[ci] (data form) or
            // W[ci] (J^H r, residual form with the BF16 Gram)
            const int roff = e < nx ? 2 * e : (resid ? rec_w(nd) : rec_z(nd)) + 2 * ci;
            constexpr int TU = 8;      // baselines whose records are in flight together
            for (int t = t0 + w; t < t1; t += TU * nw) {
                int code[TU], oth[TU];
                float2 x[TU];
#pragma unroll
                for (int u = 0; u < TU; ++u) {
                    const int tt = t + u * nw;
                    code[u] = tt < t1 ? st.ant_bl[tt] : 0;
                    const int b = code[u] >> 1;
                    oth[u] = (code[u] & 1) ? a.ant1[b] : a.ant2[b];     // the other antenna of the row
                    x[u] = make_float2(0.f, 0.f);
                    if (tt < t1) {
                        const float* rec = recs + (int64_t)b * RS + roff;
                        x[u] = make_float2(rec[0], rec[1]);
                    }
                }
#pragma unroll
                for (int u = 0; u < TU; ++u) {
                    if (t + u * nw >= t1) break;
                    const int side = code[u] & 1, o = oth[u];
                    const double2 xv = make_double2(x[u].x, side ? -x[u].y : x[u].y);
                    const float2 goc = G[ci * na + o];
                    double2 wv;
                    if (e < nx) {
                        const float2 goe = G[cj * na + o];
                        wv = make_double2((double)goc.x * goe.x + (double)goc.y * goe.y,
                                          (double)goc.y * goe.x - (double)goc.x * goe.y);   // g^ci conj(g^cj)
                    } else {
                        wv = make_double2(goc.x, goc.y);
                    }
                    const double2 pr = dmul(wv, xv);
                    acc.x += pr.x; acc.y += pr.y;
                }
            }
            part[w * 2 * WAVE + e] = acc;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
        double2 v = part[e];
        for (int w2 = 1; w2 < nw; ++w2) {
            const double2 u = part[w2 * 2 * WAVE + e];
            v.x += u.x; v.y += u.y;
        }
        if (e < nx) H[e] = v;
        else C[e - nx] = v;
    }
    __shared__ int s_fin;
    __shared__ double s_hdiag[NDMAX];
    if (threadIdx.x == 0) s_fin = 1;
    __syncthreads();
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
        const double2 v = e < nx ? H[e] : C[e - nx];
        if (!isfinite(v.x) || !isfinite(v.y)) s_fin = 0;
    }
    __syncthreads();
    const bool fin = s_fin != 0;
    bool ok = true;
    if (a.algo == WCAL_COHJONES) {
        // H = R^H R across the workgroup, right-looking: per pivot the row is scaled, then the
        // trailing triangle updated in parallel.  Every entry takes the same subtractions in
        // the same order as a serial left-looking factorisation; a pivot below
        // WCAL_EPS_PIVOT times its original diagonal (or not finite) stops it (the decision
        // reads one LDS value in every thread, so the workgroup leaves together)
        ok = fin;
        if (ok) {
            for (int i = threadIdx.x; i < nd; i += blockDim.x) s_hdiag[i] = H[tri(i, i, nd)].x;
            __syncthreads();
            for (int i = 0; i < nd; ++i) {
                const double piv = H[tri(i, i, nd)].x;
                if (!(piv > WCAL_EPS_PIVOT * s_hdiag[i]) || !isfinite(piv)) {
                    ok = false;
                    break;
                }
                const double rii = sqrt(piv);
                __syncthreads();
                for (int c = i + threadIdx.x; c < nd; c += blockDim.x) {
                    const double2 v = H[tri(i, c, nd)];
                    H[tri(i, c, nd)] = c == i ? make_double2(rii, 0.0) : make_double2(v.x / rii, v.y / rii);
                }
                __syncthreads();
                const int m = nd - i - 1;
                for (int e = threadIdx.x; e < m * (m + 1) / 2; e += blockDim.x) {
                    int r = 0, q = e;
                    while (q >= m - r) { q -= m - r; ++r; }
                    const int rr = i + 1 + r, cc = rr + q;
                    const double2 rki = H[tri(i, rr, nd)], rkj = H[tri(i, cc, nd)];
                    double2 v = H[tri(rr, cc, nd)];
                    v.x -= rki.x * rkj.x + rki.y * rkj.y;   // conj(R[i][rr]) R[i][cc]
                    v.y -= rki.x * rkj.y - rki.y * rkj.x;
                    H[tri(rr, cc, nd)] = v;
                }
                __syncthreads();
            }
        }
    }
    if (threadIdx.x == 0) {
        if (a.algo == WCAL_COHJONES) {
            if (ok) {
                chol_subst(H, C, X, nd);
                if (resid)   // g + H^-1 J^H r
                    for (int d = 0; d < nd; ++d) {
                        const float2 gd = G[d * na + p];
                        X[d] = make_double2(gd.x + X[d].x, gd.y + X[d].y);
                    }
            }
        } else {
            // AllJones: g^d + (c_d - sum_e H[d][e] g^e) / H[d][d], per direction
            for (int d = 0; d < nd; ++d) {
                const double hdd = hget(H, d, d, nd).x;
                const float2 gd = G[d * na + p];
                if (!(hdd > 0.0)) {
                    ok = false;
                    X[d] = make_double2(gd.x, gd.y);
                    continue;
                }
                double2 jr = C[d];          // with the BF16 Gram C already holds J^H r
                if (!resid)
                    for (int e = 0; e < nd; ++e) {
                        const float2 ge = G[e * na + p];
                        const double2 pr = dmul(hget(H, d, e, nd), make_double2(ge.x, ge.y));
                        jr.x -= pr.x; jr.y -= pr.y;
                    }
                X[d] = make_double2(gd.x + jr.x / hdd, gd.y + jr.y / hdd);
            }
        }
        const bool avg = avg_step(it, a.schedule);
        double dsum = 0.0, nsum = 0.0;
        float2* gn = st.gn + (int64_t)k * nd * na;
        for (int d = 0; d < nd; ++d) {
            const float2 go = G[d * na + p];
            double nr, ni;
            if (a.algo == WCAL_COHJONES && !ok) { nr = go.x; ni = go.y; }
            else { nr = X[d].x; ni = X[d].y; }
            if (avg) { nr = 0.5 * (go.x + nr); ni = 0.5 * (go.y + ni); }
            const float2 g = make_float2((float)nr, (float)ni);
            gn[d * na + p] = g;
            const double dr = (double)g.x - go.x, di = (double)g.y - go.y;
            dsum += dr * dr + di * di;
            nsum += (double)g.x * g.x + (double)g.y * g.y;
        }
        st.ant_d[(int64_t)k * na + p] = dsum;
        st.ant_n[(int64_t)k * na + p] = nsum;
        st.ant_f[(int64_t)k * na + p] = (fin ? 0 : 1) | (ok ? 0 : 2);
    }
}

// Blocks at fixed gains for the accumulate entry point.
__global__ void __launch_bounds__(DT) dd_reduce_kernel(DdArgs a, DdState st) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nd = a.n_dir, na = a.n_ant;
    const int nx = ntri(nd);
    DdSmem S = dd_smem(smem, nd, na);
    const int k = blockIdx.x;
    const float2* gk = a.gains_in + (int64_t)k * nd * na;
    for (int i = threadIdx.x; i < nd * na; i += blockDim.x) S.G[i] = gk[i];
    for (int p0 = 0; p0 < na; p0 += BA) {
        const int nb = min(BA, na - p0);
        __syncthreads();
        dd_blocks<true>(a, st, k, S.G, p0, nb, S.H, S.C, S.JR, S.CNT);
        __syncthreads();
        for (int i = threadIdx.x; i < nb * nd * nd; i += blockDim.x) {
            const int j = i / (nd * nd), c = (i / nd) % nd, e = i % nd;
            const double2 v = hget(S.H + j * nx, c, e, nd);
            a.jhj[((int64_t)k * na + p0) * nd * nd + i] = make_float2((float)v.x, (float)v.y);
        }
        for (int i = threadIdx.x; i < nb * nd; i += blockDim.x) {
            a.jhd[((int64_t)k * na + p0) * nd + i] = make_float2((float)S.C[i].x, (float)S.C[i].y);
            a.jhr[((int64_t)k * na + p0) * nd + i] = make_float2((float)S.JR[i].x, (float)S.JR[i].y);
        }
        if (a.count)
            for (int j = threadIdx.x; j < nb; j += blockDim.x) a.count[(int64_t)k * na + p0 + j] = S.CNT[j];
    }
    if (threadIdx.x == 0 && a.chi2) {
        double c = 0.0;
        for (int b = 0; b < a.n_bl; ++b) c += st.chi_bl[(int64_t)k * a.n_bl + b];
        a.chi2[k] = c;
    }
}

// Residual rows of one tile: lane <-> baseline, weights g^c_p conj(g^c_q) per round.
// PRED: the point-source model of a.pt, its phasors taken from an FP64 phase at every new time
// slot and every 16 channels, and stepped from channel to channel in between.
template <bool PRED, bool V4>
__global__ void __launch_bounds__(DT) dd_resid_kernel(DdArgs a, DdState st, int ctr_slot) {
    __shared__ double red[DT / WAVE];
    __shared__ int s_t;
    const int nd = a.n_dir, na = a.n_ant, nbl = a.n_bl;
    const bool has_flags = a.flags != nullptr;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(&st.ctr[ctr_slot], 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_t);
        if (t >= st.ntiles) break;
        const Tile T = st.tiles[t];
        const int64_t off = a.row_off[T.k];
        const float2* gk = a.gains_in + (int64_t)T.k * nd * na;
        double chi = 0.0;
        for (int b = T.b0 + threadIdx.x; b < T.b1; b += blockDim.x) {
            const int p = a.ant1[b], q = a.ant2[b];
            float2 w[NDMAX];
#pragma unroll
            for (int c = 0; c < NDMAX; ++c)
                w[c] = c < nd ? cmulc(gk[c * na + p], gk[c * na + q]) : make_float2(0.f, 0.f);
            float2 z[PRED ? NDMAX : 1], step[PRED ? NDMAX : 1];
            float part = 0.f;
            for (int s = T.s0; s < T.s1; ++s) {
                const int64_t row = off + (int64_t)s * nbl + b;
                if constexpr (PRED) {
                    const int tt = s / a.pt.n_chan, f = s - tt * a.pt.n_chan;
                    if (s == T.s0 || f % 16 == 0) {
                        const double* u = a.pt.uvw + (((int64_t)T.k * a.pt.n_time + tt) * nbl + b) * 3;
#pragma unroll
                        for (int c = 0; c < NDMAX; ++c)
                            if (c < nd) {
                                const double* l = a.pt.lmn + 3 * c;
                                const double ph = -6.283185307179586 * (u[0] * l[0] + u[1] * l[1] + u[2] * l[2]) / 299792458.0;
                                const float2 e = cis_quarter(ph * (a.pt.freq0 + f * a.pt.dfreq));
                                z[c] = make_float2(a.pt.flux[c] * e.x, a.pt.flux[c] * e.y);
                                step[c] = cis_quarter(ph * a.pt.dfreq);
                            }
                    } else {
#pragma unroll
                        for (int c = 0; c < NDMAX; ++c)
                            if (c < nd) z[c] = cmul(z[c], step[c]);
                    }
                }
                const bool fl = has_flags && a.flags[row] != 0;
                float2 r = make_float2(0.f, 0.f);
                if (!fl) {
                    r = a.data[row];
                    if constexpr (PRED) {
#pragma unroll
                        for (int c = 0; c < NDMAX; ++c)
                            if (c < nd) r = csub(r, cmul(w[c], z[c]));
                    } else {
                        // every model value of the row is requested before the first is used
                        // (indices past the last direction repeat it and are not summed); with
                        // V4 (Nd even, model 16-byte aligned) two values per 16-byte load
                        const float2* m = a.model + row * nd;
                        float2 mv[NDMAX];
                        if constexpr (V4) {
                            const float4* m4 = reinterpret_cast<const float4*>(m);
#pragma unroll
                            for (int c = 0; c < NDMAX / 2; ++c) {
                                const float4 v = m4[min(c, nd / 2 - 1)];
                                mv[2 * c] = make_float2(v.x, v.y);
                                mv[2 * c + 1] = make_float2(v.z, v.w);
                            }
                        } else {
#pragma unroll
                            for (int c = 0; c < NDMAX; ++c) mv[c] = m[min(c, nd - 1)];
                        }
#pragma unroll
                        for (int c = 0; c < NDMAX; ++c)
                            if (c < nd) r = csub(r, cmul(w[c], mv[c]));
                    }
                    part += nrm(r);
                }
                if (a.residual) a.residual[row] = r;
            }
            chi += (double)part;
        }
        chi = block_sum(chi, red);
        if (threadIdx.x == 0) st.chi_part[t] = chi;
    }
}

}  // namespace

size_t dd_stats_bytes(const wcal_problem& p) { return dd_state_bytes(p, rec_floats(p.n_dir)); }

size_t points_table_bytes(const wcal_problem& p, int32_t n_time, int32_t n_chan) {
    const size_t n = (size_t)p.n_int * n_time * p.n_bl * p.n_dir;
    const size_t nseg = ((size_t)n_chan + 63) / 64;
    return ws_round(n * nseg * 4 * sizeof(float2)) + ws_round(n * sizeof(float2));
}

size_t dd_lds_need(int nd, int na) {
    return std::max(dd_smem_size(nd, na) + kernel_static_lds(reinterpret_cast<const void*>(dd_reduce_kernel)),
                    ant_smem(nd, na) + kernel_static_lds(reinterpret_cast<const void*>(dd_ant_kernel)));
}

int dd_max_dir() { return NDMAX; }

static void launch_residual_tiles(const wcal_plan* plan, const DdArgs& a, const DdState& st, hipStream_t s,
                                  int slot) {
    const bool pred = a.pt.uvw != nullptr;
    const bool v4 = !pred && a.n_dir % 2 == 0 && reinterpret_cast<uintptr_t>(a.model) % 16 == 0;
    typedef void (*ResidFn)(DdArgs, DdState, int);
    const ResidFn fn = pred ? dd_resid_kernel<true, false> : v4 ? dd_resid_kernel<false, true> : dd_resid_kernel<false, false>;
    const int g = dd_grid(plan, reinterpret_cast<const void*>(fn), 0, st.ntiles);
    prof_begin(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(fn, dim3(g), dim3(DT), 0, s, a, st, slot);
    prof_end(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(dd_chi2_kernel, dim3((a.n_int + DT - 1) / DT), dim3(DT), 0, s, a, st);
}

hipError_t launch_dd_solve(const wcal_plan* plan, const DdArgs& a0, hipStream_t s) {
    DdArgs a = a0;
    DdState st = dd_state_of(plan, rec_floats(plan->prob.n_dir));
    const int nd = a.n_dir, na = a.n_ant;
    const int nctr = 2 * (a.max_iter + 2) + 4;
    const int64_t nblk = (int64_t)a.n_int * ((a.n_bl + GB - 1) / GB);
    const bool bf = plan->prob.precision == WCAL_PREC_BF16_GRAM;
    const bool p16 = nd % 2 == 0 && reinterpret_cast<uintptr_t>(a.model) % 16 == 0;
    typedef void (*GramFn)(DdArgs, DdState, const int32_t*, const int32_t*);
    const bool pred = a.pt.uvw != nullptr;
    GramFn gram = pred ? (a.flags ? dd_gram_pts_kernel<false> : dd_gram_pts_kernel<true>)
                       : !bf ? (p16 ? dd_gram_dmaf_kernel<16> : dd_gram_dmaf_kernel<4>) : p16 ? dd_gram_dma_kernel<16> : dd_gram_dma_kernel<4>;
    const size_t gsm = !pred && !bf ? dmaf_smem_bytes(nd) : 0;
    const int gg = dd_grid(plan, reinterpret_cast<const void*>(gram), gsm, pred ? (int64_t)a.n_int * ((a.n_bl + PGB - 1) / PGB) : nblk);
    const size_t asm_ = ant_smem(nd, na);
    prof_begin(plan, WCAL_K_OTHER, s);
    hipLaunchKernelGGL(dd_init_kernel, dim3((std::max(a.n_int, nctr) + DT - 1) / DT), dim3(DT), 0, s, a, st, 1, nctr);
    if (pred) {
        const int64_t n = (int64_t)a.n_int * a.pt.n_time * a.n_bl * nd;
        hipLaunchKernelGGL(dd_phasor_kernel, dim3((unsigned)std::min<int64_t>((n + DT - 1) / DT, 8192)), dim3(DT), 0, s, a);
    }
    prof_end(plan, WCAL_K_OTHER, s);
    const bool stats = plan->prob.mode == WCAL_MODE_STATS;
    if (stats) {
        prof_begin(plan, WCAL_K_STATS, s);
        hipLaunchKernelGGL(gram, dim3(gg), dim3(DT), gsm, s, a, st, (const int32_t*)nullptr, (const int32_t*)nullptr);
        prof_end(plan, WCAL_K_STATS, s);
    }
    for (int it = 0; it < a.max_iter; ++it) {
        DdState sti = st;
        sti.ctr = st.ctr + dd_pop_slot(it);      // Gram pops of this update at sti.ctr[0]
        if (!stats) {
            const int32_t* lst = it == 0 ? nullptr : st.alist + (it & 1) * a.n_int;
            prof_begin(plan, WCAL_K_PASS, s);
            const int32_t* nl = st.ctr + dd_nlist_slot(it);
            hipLaunchKernelGGL(gram, dim3(gg), dim3(DT), gsm, s, a, sti, lst, nl);
            prof_end(plan, WCAL_K_PASS, s);
        }
        prof_begin(plan, stats ? WCAL_K_SOLVE_STATS : WCAL_K_UPDATE, s);
        hipLaunchKernelGGL(dd_ant_kernel, dim3(a.n_int * na), dim3(DT), asm_, s, a, st, it);
        hipLaunchKernelGGL(dd_finish_kernel, dim3(a.n_int), dim3(DT), 0, s, a, st, it);
        prof_end(plan, stats ? WCAL_K_SOLVE_STATS : WCAL_K_UPDATE, s);
        if (watch_stop(plan, s, st.ctr + dd_nlist_slot(it + 1), it)) break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.residual || a.chi2) {
        a.gains_in = a.gains;
        launch_residual_tiles(plan, a, st, s, nctr - 1);
    }
    return hipGetLastError();
}

hipError_t launch_dd_accumulate(const wcal_plan* plan, const DdArgs& a, hipStream_t s) {
    DdState st = dd_state_of(plan, rec_floats(plan->prob.n_dir));
    const int nd = a.n_dir, na = a.n_ant;
    const int nctr = 4;
    hipLaunchKernelGGL(dd_init_kernel, dim3(1), dim3(DT), 0, s, a, st, 0, nctr);
    const int64_t ntask = (int64_t)a.n_int * a.n_bl;
    const int gg = dd_grid(plan, reinterpret_cast<const void*>(dd_gram_kernel<true>), 0, (ntask + 3) / 4);
    hipLaunchKernelGGL(dd_gram_kernel<true>, dim3(gg), dim3(DT), 0, s, a, st, 0);
    hipLaunchKernelGGL(dd_reduce_kernel, dim3(a.n_int), dim3(DT), dd_smem_size(nd, na), s, a, st);
    return hipGetLastError();
}

hipError_t launch_dd_residual(const wcal_plan* plan, const DdArgs& a, hipStream_t s) {
    DdState st = dd_state_of(plan, rec_floats(plan->prob.n_dir));
    hipLaunchKernelGGL(dd_init_kernel, dim3(1), dim3(DT), 0, s, a, st, 0, 4);
    launch_residual_tiles(plan, a, st, s, 3);
    return hipGetLastError();
}
