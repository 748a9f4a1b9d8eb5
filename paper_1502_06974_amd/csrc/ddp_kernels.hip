// Direction-dependent kernels for gfx950 with 2x2 Jones gains (Sect. 4.4): polarized
// CohJones (separable by antenna: per-antenna blocks inverted exactly) and polarized
// AllJones (separable by antenna and direction, residual form, Eq. update:DD:diag:pol).
//
// Normal equations.  With Y^d_pq = M^d_pq G^{dH}_q stacked over directions into Ys
// [2Nd x 2] (row 2d + k = row k of Y^d), the model of a row is the 2 x 2Nd matrix of the
// stacked gains [G^0 .. G^{Nd-1}] times Ys.  The operator-diagonal block of Eq. JHJ:DD:pol
// for antenna p therefore acts on both rows of the gains alike, as G -> G H_p with
//     H_p = sum Ys Ys^H        (2Nd x 2Nd Hermitian; block (c, e) = sum Y^c Y^{eH}),
// and the top half of J^H D (Eq. JHR:DD:pol with D for R) is N_p = sum D Ys^H (2 x 2Nd).
// CohJones solves G H_p = N_p (one 2Nd Cholesky, two right-hand sides); AllJones takes
// G^d + J^H r^d (H_p^{dd})^-1 per direction with J^H r = N_p - G H_p.
//
// Gram pass (MFMA): the gains factor out of the sums over samples.  Per baseline the pass
// forms the Hermitian Gram of the per-sample vector x = [vec M^0 .. vec M^{Nd-1} | vec D]
// (4 Nd + 4 complex; vec index 2 i + k of entry (i, k)), Gram[x][y] = sum conj(x) y, and the
// contraction with the gains of the other antenna o of each row gives
//   row pq (p = ant1):  H[2c+k][2e+l] += sum_ab W^ce[a][b] conj(Gram[4c+2k+a][4e+2l+b])
//                       N[i][2e+l]    += sum_jb G^e_o[j][b] Gram[4e+2l+b][4Nd+2i+j]
//   row qp (p = ant2):  H[2c+k][2e+l] += sum_ab W^ce[a][b] Gram[4c+2a+k][4e+2b+l]
//                       N[i][2e+l]    += sum_jb G^e_o[j][b] conj(Gram[4e+2b+l][4Nd+2j+i])
// with W^ce = G^{cH}_o G^e_o.  Lane l of a wavefront holds column l % 16 of sample l / 16;
// each v_mfma_f32_16x16x4f32 consumes 4 samples.  The complex Gram is formed in a real
// embedding: a diagonal 16-column tile takes three MFMAs (Re = Ar^T Ar + Ai^T Ai,
// T = Ar^T Ai, Im = T - T^T), an off-diagonal tile pair three by Gauss's product
// (T1 = Ar^T Br, T2 = Ai^T Bi, T3 = (Ar + Ai)^T (Br - Bi); Re = T1 + T2,
// Im = T1 - T2 - T3), 18 MFMAs per 4 samples at three tiles instead of 21.  Flagged
// samples enter as zeros (selected, not multiplied).
// The accumulate pass adds four residual columns vec R, R = D - sum_d G^d_p M^d G^{dH}_q
// formed per sample in the pass, whose products with the model columns give J^H r.
#include "dd_common.h"

using namespace wcal_dev;

namespace {

constexpr int PND = 10;   // directions: 4 (Nd + 2) columns fit three 16-wide tiles
constexpr int PGB = 4;    // baselines per workgroup task (one per wavefront)
constexpr int PGS = 16;   // samples per chunk

// per-sample columns [M | D]
__host__ __device__ inline int pcols(int nd) { return 4 * nd + 4; }
// record floats: upper triangle of the [M | D] Gram (complex, packed row-major), then
// W [4 Nd][4] = sum conj(M) R (accumulate pass), then the unflagged-sample count
__host__ __device__ inline int prec_w(int nd) { return 2 * ntri(pcols(nd)); }
__host__ __device__ inline int prec_cnt(int nd) { return prec_w(nd) + 32 * nd; }
__host__ __device__ inline int prec_floats(int nd) { return (prec_cnt(nd) + 1 + 3) / 4 * 4; }
// 16-column tiles of the pass: [M | D] (solve) or [M | D | R] (accumulate)
inline int ptiles(int nd, bool with_r) { return (4 * nd + (with_r ? 8 : 4) + 15) / 16; }

// outputs of the per-antenna contraction: H (packed upper), N, and J^H r (accumulate)
__host__ __device__ inline int pn_h(int nd) { return ntri(2 * nd); }
__host__ __device__ inline int pn_n(int nd) { return 4 * nd; }
constexpr int PNOUT = (2 * PND) * (2 * PND + 1) / 2 + 2 * 4 * PND;   // 290
constexpr int PMCH = 256;   // rows of an antenna whose metadata is staged at once
// LDS bytes of the gains [nd][na][4], rounded up to 16
__host__ __device__ inline size_t pg_bytes(int nd, int na) { return (size_t)nd * na * 4 * sizeof(float2); }
inline size_t pant_smem(int nd, int na) {
    return pg_bytes(nd, na) + ((size_t)(DT / WAVE) * PNOUT + pn_h(nd) + 4 * pn_n(nd)) * sizeof(double2) +
           2 * (size_t)PMCH * sizeof(int);
}

// ------------------------------------------------------------------ Gram pass
// A workgroup owns PGB consecutive baselines of one interval and walks its samples in
// chunks of PGS.  For each sample the model rows of the PGB baselines are one contiguous
// segment (PGB * 4 Nd complex) and their data rows another (PGB * 4), so a chunk is read
// as 16-byte pieces with consecutive addresses across the workgroup, staged in registers
// while the previous chunk is consumed, and laid out in LDS as [sample][baseline][column].
// Wavefront w runs the MFMAs of baseline w: per chunk it reads its operands of all four
// 4-sample groups from LDS at once, then issues the first product into every accumulator
// before any second one, so dependent MFMAs stay a dozen apart.
constexpr int PQPT = (PGS * PGB * (4 * PND + 4) / 2 + DT - 1) / DT;   // staged float4 per thread

template <int NT, bool WITH_R>
__device__ __forceinline__ void ddp_gram_body(const DdArgs& a, const DdState& st, const int32_t* list,
                                              const int32_t* n_list) {
    constexpr int W16 = 16 * NT;
    __shared__ __align__(16) float2 abuf[PGS][PGB][W16];
    __shared__ uint8_t fbuf[PGS][PGB];
    __shared__ int s_task;
    __shared__ double chs[WITH_R ? DT : 1];
    extern __shared__ __align__(16) float2 gsh[];     // accumulate: gains [nd][na][4]
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int nd = a.n_dir, nbl = a.n_bl, na = a.n_ant;
    const int nm = 4 * nd, ncs = nm + 4, nct = WITH_R ? ncs + 4 : ncs;
    const int RS = prec_floats(nd);
    const int kk = lane >> 4, col = lane & 15;
    const int nbb = (nbl + PGB - 1) / PGB;
    const int nint = list ? *n_list : a.n_int;
    const int64_t ntask = (int64_t)nint * nbb;
    if ((int64_t)blockIdx.x >= ntask) return;   // tasks are popped dynamically
    const bool has_flags = a.flags != nullptr;
    // static decode of this thread's staged pieces: offset in float4 from the chunk's first
    // model (or data) row, and a code (LDS float4 slot | sample << 11 | baseline << 15 |
    // data << 17; -1 for no piece)
    const int qm = PGB * nm / 2, qd = PGB * 2;   // float4 per sample: model, data
    int goff[PQPT], code[PQPT];
#pragma unroll
    for (int r = 0; r < PQPT; ++r) {
        const int q = threadIdx.x + DT * r;
        goff[r] = 0;
        code[r] = -1;
        if (q < PGS * (qm + qd)) {
            const int sm = q / (qm + qd), rem = q % (qm + qd);
            if (rem < qm) {
                const int bl = 2 * rem / nm, c = 2 * rem % nm;
                goff[r] = sm * nbl * (nm / 2) + rem;
                code[r] = (((sm * PGB + bl) * W16 + c) >> 1) | (sm << 11) | (bl << 15);
            } else {
                const int dq = rem - qm, bl = dq >> 1, c = nm + 2 * (dq & 1);
                goff[r] = sm * nbl * 2 + dq;
                code[r] = (((sm * PGB + bl) * W16 + c) >> 1) | (sm << 11) | (bl << 15) | (1 << 17);
            }
        }
    }
    const int fs = threadIdx.x / PGB, fb = threadIdx.x % PGB;   // flag staged by this thread
    const bool fown = threadIdx.x < PGS * PGB;
    float4* lds4 = reinterpret_cast<float4*>(&abuf[0][0][0]);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_task = atomicAdd(&st.ctr[0], 1);
        __syncthreads();
        const int task = __builtin_amdgcn_readfirstlane(s_task);
        if (task >= ntask) break;
        const int k = list ? list[task / nbb] : a.order[task / nbb];
        const int b0 = (task % nbb) * PGB;
        const int64_t off = a.row_off[k];
        const int ns = a.ns[k];
        const int nch = (ns + PGS - 1) / PGS;
        if constexpr (WITH_R) {
            const float2* gk = a.gains_in + (int64_t)k * nd * na * 4;
            for (int i = threadIdx.x; i < nd * na * 4; i += DT) gsh[i] = gk[i];
        }
        float4 stage[PQPT];
        uint8_t fstage = 1;
        auto fetch = [&](int c) {
            const int s0 = c * PGS;
            const int64_t row0 = off + (int64_t)s0 * nbl + b0;
            const float4* mb = reinterpret_cast<const float4*>(a.model) + row0 * (nm / 2);
            const float4* db = reinterpret_cast<const float4*>(a.data) + row0 * 2;
#pragma unroll
            for (int r = 0; r < PQPT; ++r) {
                const int cd = code[r];
                const bool ok = cd >= 0 && s0 + ((cd >> 11) & 15) < ns && b0 + ((cd >> 15) & 3) < nbl;
                stage[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (ok) stage[r] = (cd >> 17) ? load_at(db, goff[r]) : load_at(mb, goff[r]);
            }
            const bool fok = fown && s0 + fs < ns && b0 + fb < nbl;
            fstage = 1;
            if (fok) fstage = has_flags ? (uint8_t)(a.flags[row0 + (int64_t)fs * nbl + fb] != 0) : (uint8_t)0;
        };
        constexpr int NO = NT * (NT - 1) / 2 + 1;
        floatx4 dre[NT], dti[NT], ot1[NO], ot2[NO], ot3[NO];   // diagonal: Re, T; off-diagonal: T1, T2, T3
#pragma unroll
        for (int t = 0; t < NT; ++t) { dre[t] = floatx4{0.f, 0.f, 0.f, 0.f}; dti[t] = dre[t]; }
#pragma unroll
        for (int t = 0; t < NO; ++t) { ot1[t] = floatx4{0.f, 0.f, 0.f, 0.f}; ot2[t] = ot1[t]; ot3[t] = ot1[t]; }
        int cnt = 0;
        double chi = 0.0;
        fetch(0);
        for (int c = 0; c < nch; ++c) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < PQPT; ++r)
                if (code[r] >= 0) lds4[code[r] & 2047] = stage[r];
            if (fown) fbuf[fs][fb] = fstage;
            __syncthreads();
            if (c + 1 < nch) fetch(c + 1);
            if constexpr (WITH_R) {
                // R = D - sum_d G^d_p M^d G^{dH}_q, one entry (i, j) per thread
                const int pr = threadIdx.x >> 2, sm = pr / PGB, bl = pr % PGB;
                const int e = threadIdx.x & 3, i = e >> 1, j = e & 1;
                const int b = b0 + bl, s = c * PGS + sm;
                float2 r = make_float2(0.f, 0.f);
                const bool valid = s < ns && b < nbl;
                if (valid && !fbuf[sm][bl]) {
                    const int p = a.ant1[b], q = a.ant2[b];
                    r = abuf[sm][bl][nm + e];
                    for (int d = 0; d < nd; ++d) {
                        const float2* gp = gsh + (d * na + p) * 4;
                        const float2* gq = gsh + (d * na + q) * 4;
                        const float2* mm = &abuf[sm][bl][4 * d];
#pragma unroll
                        for (int kx = 0; kx < 2; ++kx) {
                            // (M G_q^H)[kx][j] = sum_l M[kx][l] conj(G_q[j][l])
                            const float2 t = cadd(cmulc(mm[2 * kx], gq[2 * j]), cmulc(mm[2 * kx + 1], gq[2 * j + 1]));
                            r = csub(r, cmul(gp[2 * i + kx], t));
                        }
                    }
                    chi += (double)nrm(r);
                }
                if (valid && a.residual) a.residual[(off + (int64_t)s * nbl + b) * 4 + e] = r;
                __syncthreads();
                abuf[sm][bl][ncs + e] = r;
                __syncthreads();
            }
            constexpr int NG = PGS / 4;
            float2 v[NG][NT];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int sl = 4 * g + kk;
                const bool use = !fbuf[sl][w];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int cc = 16 * t + col;
                    v[g][t] = (use && cc < nct) ? abuf[sl][w][cc] : make_float2(0.f, 0.f);
                }
                if (use && col == 0) ++cnt;
            }
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                // first products into every accumulator, then the second ones
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    dre[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[g][t].x, v[g][t].x, dre[t], 0, 0, 0);
                    dti[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[g][t].x, v[g][t].y, dti[t], 0, 0, 0);
                }
                {
                    int o = 0;
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int u = t + 1; u < NT; ++u, ++o) {
                            ot1[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[g][t].x, v[g][u].x, ot1[o], 0, 0, 0);
                            ot2[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[g][t].y, v[g][u].y, ot2[o], 0, 0, 0);
                            ot3[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[g][t].x + v[g][t].y, v[g][u].x - v[g][u].y, ot3[o], 0, 0, 0);
                        }
                }
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    dre[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[g][t].y, v[g][t].y, dre[t], 0, 0, 0);
            }
        }
        // epilogue: the record of the wavefront's baseline; the diagonal tiles go through the
        // wavefront's own 2 x 256 floats of the (now free) staging buffer
        __syncthreads();
        float* tile = reinterpret_cast<float*>(&abuf[0][0][0]) + w * 512;
        // entry (c1, c2), c1 <= c2, of the Gram: [M | D] block or the W block
        auto put = [&](float* rec, int c1, int c2, float re, float im) {
            if (c2 < ncs) {
                const int t = tri(c1, c2, ncs);
                rec[2 * t] = re;
                rec[2 * t + 1] = im;
            } else if (WITH_R && c2 < ncs + 4 && c1 < nm) {
                const int t = prec_w(nd) + 2 * (4 * c1 + (c2 - ncs));
                rec[t] = re;
                rec[t + 1] = im;
            }
        };
        {
            const int b = b0 + w;
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, WAVE);
            float* rec = st.rec + ((int64_t)k * nbl + b) * RS;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * (lane >> 4) + r;
                    tile[i * 16 + col] = dre[t][r];
                    tile[256 + i * 16 + col] = dti[t][r];
                }
                __builtin_amdgcn_wave_barrier();
                if (b < nbl)
                    for (int e = lane; e < 256; e += WAVE) {
                        const int i = e >> 4, jj = e & 15;
                        if (i <= jj && 16 * t + jj < nct)
                            put(rec, 16 * t + i, 16 * t + jj, tile[i * 16 + jj],
                                tile[256 + i * 16 + jj] - tile[256 + jj * 16 + i]);
                    }
                __builtin_amdgcn_wave_barrier();
            }
            if (b < nbl) {
                int o = 0;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int u = t + 1; u < NT; ++u, ++o)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int c1 = 16 * t + 4 * (lane >> 4) + r, c2 = 16 * u + col;
                            if (c2 < nct) put(rec, c1, c2, ot1[o][r] + ot2[o][r], ot1[o][r] - ot2[o][r] - ot3[o][r]);
                        }
                if (lane == 0) reinterpret_cast<int*>(rec)[prec_cnt(nd)] = cnt;
            }
        }
        if constexpr (WITH_R) {
            // chi^2 per baseline: the threads of baseline bl are those with (tid / 4) % PGB == bl
            chs[threadIdx.x] = chi;
            __syncthreads();
            if ((int)threadIdx.x < PGB && b0 + (int)threadIdx.x < nbl) {
                double c = 0.0;
                for (int t = 4 * threadIdx.x; t < DT; t += 4 * PGB)
                    for (int e = 0; e < 4; ++e) c += chs[t + e];
                st.chi_bl[(int64_t)k * nbl + b0 + threadIdx.x] = c;
            }
        }
    }
}

template <int NT>
__global__ void __launch_bounds__(DT) __attribute__((amdgpu_waves_per_eu(3, 8))) ddp_gram_kernel(DdArgs a, DdState st, const int32_t* list,
                                                      const int32_t* n_list) {
    ddp_gram_body<NT, false>(a, st, list, n_list);
}

template <int NT>
__global__ void __launch_bounds__(DT) ddp_gram_r_kernel(DdArgs a, DdState st) {
    ddp_gram_body<NT, true>(a, st, nullptr, nullptr);
}

// ------------------------------------------------------------------ per-antenna update
__device__ __forceinline__ double2 dcmulc(double2 a, double2 b) {   // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 d2(float2 a) { return make_double2(a.x, a.y); }

// H[i][j] of a packed upper triangle (any i, j)
__device__ __forceinline__ double2 phget(const double2* h, int i, int j, int n) {
    return i <= j ? h[tri(i, j, n)] : dconj(h[tri(j, i, n)]);
}

// One workgroup per (interval, antenna).  Contraction: lanes run over the outputs (H packed
// upper, N, and J^H r when accumulating), the four wavefronts take every fourth of the
// antenna's baselines in CSR order (record offset, side and other antenna staged in LDS
// once), two baselines' record loads in flight per lane; the wavefronts' FP64 sums are
// folded in wavefront order.
// Solve mode, in FP64: CohJones factors H = R^H R across the workgroup (right-looking: one
// pivot per step, then the trailing triangle in parallel) and one thread per row of the
// gains substitutes; AllJones forms J^H r = N - G H and the per-direction 2x2 steps in
// parallel.  The schedule is applied per gain entry, and the FP64 relative-change norms
// are summed in a fixed order.  Accumulate mode writes the blocks instead.
template <bool ACC>
__global__ void __launch_bounds__(DT) ddp_ant_kernel(DdArgs a, DdState st, int it) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[DT / WAVE];
    __shared__ double hdiag[2 * PND];
    __shared__ int s_bad;      // 1: non-finite blocks, 2: singular block
    const int nd = a.n_dir, na = a.n_ant, nbl = a.n_bl;
    const int n2 = 2 * nd, nm = 4 * nd, ncs = nm + 4;
    const int nh = pn_h(nd), nn = pn_n(nd);
    const int nout = nh + nn * (ACC ? 2 : 1);
    const int nw = DT / WAVE;
    const int k = blockIdx.x / na, p = blockIdx.x % na;
    if (!ACC && !st.active[k]) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    float2* G = reinterpret_cast<float2*>(smem);                             // [nd][na][4]
    double2* part = reinterpret_cast<double2*>(smem + pg_bytes(nd, na));    // [nw][PNOUT]
    double2* H = part + nw * PNOUT;    // [nh]
    double2* N = H + nh;               // [2][n2]
    double2* JR = N + nn;              // [2][n2]
    double2* X = JR + nn;              // [2][n2]
    double2* S = part;                 // [n2][n2] Cholesky factor (after the fold)
    const float2* gk = (ACC ? a.gains_in : a.gains) + (int64_t)k * nd * na * 4;
    for (int i = threadIdx.x; i < nd * na * 4; i += DT) G[i] = gk[i];
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const int RS = prec_floats(nd);
    const float* recs = st.rec + (int64_t)k * nbl * RS;
    const int t0 = st.ant_ptr[p], t1 = st.ant_ptr[p + 1];
    // the antenna's rows, staged in LDS in chunks of PMCH: record offset, and
    // side | other antenna << 1 (chunk starts are multiples of the wavefront count, so each
    // wavefront sums the same rows in the same order whatever the chunking)
    int* meta = reinterpret_cast<int*>(X + nn);     // [2 PMCH]
    for (int e = lane; e < nout; e += WAVE) part[w * PNOUT + e] = make_double2(0.0, 0.0);
    for (int base = t0; base < t1; base += PMCH) {
        const int nt = min(PMCH, t1 - base);
        __syncthreads();
        for (int t = threadIdx.x; t < nt; t += DT) {
            const int code = st.ant_bl[base + t];
            const int b = code >> 1, side = code & 1;
            meta[2 * t] = b * RS;
            meta[2 * t + 1] = side | ((side ? a.ant1[b] : a.ant2[b]) << 1);
        }
        __syncthreads();
        for (int e = lane; e < nout; e += WAVE) {
            double2 acc = part[w * PNOUT + e];
            if (e < nh) {
                int r1 = 0, rem = e;
                while (rem >= n2 - r1) { rem -= n2 - r1; ++r1; }
                const int r2 = r1 + rem;
                const int c = r1 >> 1, kr = r1 & 1, ee = r2 >> 1, l = r2 & 1;
#pragma unroll 2
                for (int t = w; t < nt; t += nw) {
                    const int side = meta[2 * t + 1] & 1, o = meta[2 * t + 1] >> 1;
                    const float* rec = recs + meta[2 * t];
                    // H[2c+kr][2ee+l] += sum_ab W^{c,ee}[a][b] x_ab, W = G^{cH}_o G^{ee}_o
                    float2 x[4];
#pragma unroll
                    for (int ab = 0; ab < 4; ++ab) {
                        const int aa = ab >> 1, bb = ab & 1;
                        const int xi = side ? 4 * c + 2 * aa + kr : 4 * c + 2 * kr + aa;
                        const int yi = side ? 4 * ee + 2 * bb + l : 4 * ee + 2 * l + bb;
                        // stored (min, max); conjugate when swapped, and once more on side 0
                        const float* q = rec + 2 * (xi <= yi ? tri(xi, yi, ncs) : tri(yi, xi, ncs));
                        const bool cj = (xi > yi) != (side == 0);
                        x[ab] = make_float2(q[0], cj ? -q[1] : q[1]);
                    }
                    const float2* gc = G + (c * na + o) * 4;
                    const float2* ge = G + (ee * na + o) * 4;
#pragma unroll
                    for (int ab = 0; ab < 4; ++ab) {
                        const int aa = ab >> 1, bb = ab & 1;
                        const double2 w0 = dcmulc(d2(gc[aa]), d2(ge[bb]));
                        const double2 w1 = dcmulc(d2(gc[2 + aa]), d2(ge[2 + bb]));
                        const double2 pr = dmul(make_double2(w0.x + w1.x, w0.y + w1.y), d2(x[ab]));
                        acc.x += pr.x; acc.y += pr.y;
                    }
                }
            } else {
                const int f = e - nh;
                const bool jr = f >= nn;
                const int idx = jr ? f - nn : f;
                const int i = idx / n2, cc = idx % n2, ee = cc >> 1, l = cc & 1;
#pragma unroll 2
                for (int t = w; t < nt; t += nw) {
                    const int side = meta[2 * t + 1] & 1, o = meta[2 * t + 1] >> 1;
                    const float* rec = recs + meta[2 * t];
                    // N[i][2ee+l] (or J^H r) += sum_jb G^{ee}_o[j][b] x_jb
                    float2 x[4];
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb) {
                        const int j = jb >> 1, bb = jb & 1;
                        const int xi = side ? 4 * ee + 2 * bb + l : 4 * ee + 2 * l + bb;
                        const int yi = side ? 2 * j + i : 2 * i + j;
                        const float* q = jr ? rec + prec_w(nd) + 2 * (4 * xi + yi) : rec + 2 * tri(xi, nm + yi, ncs);
                        x[jb] = make_float2(q[0], side ? -q[1] : q[1]);
                    }
                    const float2* ge = G + (ee * na + o) * 4;
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb) {
                        const double2 pr = dmul(d2(ge[jb]), d2(x[jb]));
                        acc.x += pr.x; acc.y += pr.y;
                    }
                }
            }
            part[w * PNOUT + e] = acc;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nout; e += DT) {
        double2 v = part[e];
        for (int w2 = 1; w2 < nw; ++w2) {
            const double2 u = part[w2 * PNOUT + e];
            v.x += u.x; v.y += u.y;
        }
        H[e] = v;     // H, then N, then JR: contiguous
    }
    __syncthreads();
    if constexpr (ACC) {
        const int64_t ap = (int64_t)k * na + p;
        for (int i = threadIdx.x; i < n2 * n2; i += DT) {
            const double2 v = phget(H, i / n2, i % n2, n2);
            a.jhj[ap * n2 * n2 + i] = make_float2((float)v.x, (float)v.y);
        }
        // jhd / jhr [d][2 i + l] = N[i][2 d + l]
        for (int i = threadIdx.x; i < nn; i += DT) {
            const int d = i >> 2, r = (i >> 1) & 1, l = i & 1;
            const double2 v = N[r * n2 + 2 * d + l], u = JR[r * n2 + 2 * d + l];
            a.jhd[ap * nn + i] = make_float2((float)v.x, (float)v.y);
            a.jhr[ap * nn + i] = make_float2((float)u.x, (float)u.y);
        }
        if (threadIdx.x == 0 && a.count) {
            int c = 0;
            for (int t = t0; t < t1; ++t)
                c += reinterpret_cast<const int*>(recs + (int64_t)(st.ant_bl[t] >> 1) * RS)[prec_cnt(nd)];
            a.count[ap] = c;
        }
        return;
    }
    {
        bool f = true;
        for (int i = threadIdx.x; i < nh + nn; i += DT) f = f && isfinite(H[i].x) && isfinite(H[i].y);
        if (!f) atomicOr(&s_bad, 1);
    }
    __syncthreads();
    const bool fin = !(s_bad & 1);
    // stacked gains of this antenna: Gs[i][2 d + l] = G^d[i][l]
    auto gs = [&](int i, int cc) { return d2(G[((cc >> 1) * na + p) * 4 + 2 * i + (cc & 1)]); };
    if (a.algo == WCAL_COHJONES) {
        if (fin) {
            for (int e = threadIdx.x; e < n2 * n2; e += DT) {
                const int r = e / n2, c = e % n2;
                S[e] = r <= c ? H[tri(r, c, n2)] : make_double2(0.0, 0.0);
            }
            for (int i = threadIdx.x; i < n2; i += DT) hdiag[i] = H[tri(i, i, n2)].x;
            __syncthreads();
            for (int i = 0; i < n2; ++i) {
                const double piv = S[i * n2 + i].x;
                if (!(piv > WCAL_EPS_PIVOT * hdiag[i]) || !isfinite(piv)) {   // same value in every thread
                    if (threadIdx.x == 0) s_bad |= 2;
                    break;
                }
                const double rii = sqrt(piv);
                __syncthreads();
                for (int c = i + threadIdx.x; c < n2; c += DT) {
                    const double2 v = S[i * n2 + c];
                    S[i * n2 + c] = c == i ? make_double2(rii, 0.0) : make_double2(v.x / rii, v.y / rii);
                }
                __syncthreads();
                // trailing triangle: S[r][c] -= conj(R[i][r]) R[i][c], i < r <= c
                const int mrem = n2 - i - 1;
                for (int e = threadIdx.x; e < mrem * (mrem + 1) / 2; e += DT) {
                    int r = 0, q = e;
                    while (q >= mrem - r) { q -= mrem - r; ++r; }
                    const int rr = i + 1 + r, cc = rr + q;
                    const double2 pr = dcmulc(S[i * n2 + rr], S[i * n2 + cc]);
                    S[rr * n2 + cc].x -= pr.x;
                    S[rr * n2 + cc].y -= pr.y;
                }
                __syncthreads();
            }
            __syncthreads();
            if (!(s_bad & 2) && threadIdx.x < 2) {
                // row i of G H = N: H x = conj(row i of N), row i of G = conj(x)
                const int i = threadIdx.x;
                double2* x = X + i * n2;
                for (int r = 0; r < n2; ++r) {          // R^H z = conj(N_i)
                    double2 v = dconj(N[i * n2 + r]);
                    for (int q = 0; q < r; ++q) {
                        const double2 pr = dcmulc(S[q * n2 + r], x[q]);
                        v.x -= pr.x; v.y -= pr.y;
                    }
                    const double d = S[r * n2 + r].x;
                    x[r] = make_double2(v.x / d, v.y / d);
                }
                for (int r = n2 - 1; r >= 0; --r) {     // R x = z
                    double2 v = x[r];
                    for (int q = r + 1; q < n2; ++q) {
                        const double2 pr = dmul(S[r * n2 + q], x[q]);
                        v.x -= pr.x; v.y -= pr.y;
                    }
                    const double d = S[r * n2 + r].x;
                    x[r] = make_double2(v.x / d, v.y / d);
                }
                for (int r = 0; r < n2; ++r) x[r] = dconj(x[r]);
            }
        }
    } else {
        // AllJones: J^H r = N - G H, then G^d + (J^H r)^d (H^dd)^-1 per direction
        for (int e = threadIdx.x; e < nn; e += DT) {
            const int i = e / n2, cc = e % n2;
            double2 v = N[e];
            for (int c2 = 0; c2 < n2; ++c2) {
                const double2 pr = dmul(gs(i, c2), phget(H, c2, cc, n2));
                v.x -= pr.x; v.y -= pr.y;
            }
            JR[e] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n2; e += DT) {
            const int d = e >> 1, i = e & 1;
            const double z00 = H[tri(2 * d, 2 * d, n2)].x, z11 = H[tri(2 * d + 1, 2 * d + 1, n2)].x;
            const double2 z01 = H[tri(2 * d, 2 * d + 1, n2)];
            const double det = z00 * z11 - (z01.x * z01.x + z01.y * z01.y);
            const bool sing = !(z00 > 0.0) || !(det > WCAL_EPS_PIVOT * z00 * z11);
            const double2 j0 = JR[i * n2 + 2 * d], j1 = JR[i * n2 + 2 * d + 1];
            const double2 g0 = gs(i, 2 * d), g1 = gs(i, 2 * d + 1);
            if (sing) atomicOr(&s_bad, 2);
            if (sing || !fin) {
                X[i * n2 + 2 * d] = g0;
                X[i * n2 + 2 * d + 1] = g1;
                continue;
            }
            // Z^-1 = [[z11, -z01], [-conj(z01), z00]] / det
            const double2 a0 = dmul(j1, dconj(z01)), a1 = dmul(j0, z01);
            X[i * n2 + 2 * d] = make_double2(g0.x + (j0.x * z11 - a0.x) / det, g0.y + (j0.y * z11 - a0.y) / det);
            X[i * n2 + 2 * d + 1] = make_double2(g1.x + (j1.x * z00 - a1.x) / det, g1.y + (j1.y * z00 - a1.y) / det);
        }
    }
    __syncthreads();
    const bool ok = !(s_bad & 2);
    const bool keep = a.algo == WCAL_COHJONES && (!ok || !fin);
    const bool avg = avg_step(it, a.schedule);
    double dsum = 0.0, nsum = 0.0;
    float2* gn = st.gn + (int64_t)k * nd * na * 4;
    for (int e = threadIdx.x; e < nn; e += DT) {
        const int d = e >> 2, i = (e >> 1) & 1, l = e & 1;
        const double2 go = gs(i, 2 * d + l);
        double2 v = keep ? go : X[i * n2 + 2 * d + l];
        if (avg) v = make_double2(0.5 * (go.x + v.x), 0.5 * (go.y + v.y));
        const float2 g = make_float2((float)v.x, (float)v.y);
        gn[(d * na + p) * 4 + 2 * i + l] = g;
        const double dr = (double)g.x - go.x, di = (double)g.y - go.y;
        dsum += dr * dr + di * di;
        nsum += (double)g.x * g.x + (double)g.y * g.y;
    }
    dsum = block_sum(dsum, red);
    nsum = block_sum(nsum, red);
    if (threadIdx.x == 0) {
        st.ant_d[(int64_t)k * na + p] = dsum;
        st.ant_n[(int64_t)k * na + p] = nsum;
        st.ant_f[(int64_t)k * na + p] = (fin ? 0 : 1) | (ok ? 0 : 2);
    }
}

// chi^2 per interval from the accumulate pass's per-baseline sums, in baseline order
__global__ void __launch_bounds__(DT) ddp_chi2_bl_kernel(DdArgs a, DdState st) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_int || !a.chi2) return;
    double c = 0.0;
    for (int b = 0; b < a.n_bl; ++b) c += st.chi_bl[(int64_t)k * a.n_bl + b];
    a.chi2[k] = c;
}

// ------------------------------------------------------------------ residual pass
// Persistent over the plan's tiles; per tile the interval's gains are staged in LDS and
// lane <-> baseline walks the tile's samples: R = D - sum_d G^d_p M^d G^{dH}_q.
constexpr int RB = 10;   // directions loaded together: PND, one batch (as a loop: 151 VGPRs; as one block: 180)
__global__ void __launch_bounds__(DT) ddp_resid_kernel(DdArgs a, DdState st, int ctr_slot) {
    extern __shared__ __align__(16) float2 gsh[];
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
        const float2* gk = a.gains_in + (int64_t)T.k * nd * na * 4;
        for (int i = threadIdx.x; i < nd * na * 4; i += DT) gsh[i] = gk[i];
        __syncthreads();
        double chi = 0.0;
        for (int b = T.b0 + threadIdx.x; b < T.b1; b += blockDim.x) {
            const int p = a.ant1[b], q = a.ant2[b];
            float part = 0.f;
            for (int s = T.s0; s < T.s1; ++s) {
                const int64_t row = off + (int64_t)s * nbl + b;
                const bool fl = has_flags && a.flags[row] != 0;
                J2 R = J2{make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                if (!fl) {
                    R = load_j2(a.data, row);
                    // the model blocks of RB directions are all requested before the first is
                    // used (indices past the last direction repeat it and are not summed)
                    for (int d0 = 0; d0 < nd; d0 += RB) {
                        J2 M[RB];
#pragma unroll
                        for (int u = 0; u < RB; ++u) M[u] = load_j2(a.model, row * nd + min(d0 + u, nd - 1));
#pragma unroll
                        for (int u = 0; u < RB; ++u) {
                            if (d0 + u < nd) {
                                const float2* gp = gsh + ((d0 + u) * na + p) * 4;
                                const float2* gq = gsh + ((d0 + u) * na + q) * 4;
                                const J2 Gp{gp[0], gp[1], gp[2], gp[3]}, Gq{gq[0], gq[1], gq[2], gq[3]};
                                R = jsub(R, mulH(mul(Gp, M[u]), Gq));
                            }
                        }
                    }
                    part += nrm(R.a) + nrm(R.b) + nrm(R.c) + nrm(R.d);
                }
                if (a.residual) store_j2(a.residual, row, R);
            }
            chi += (double)part;
        }
        chi = block_sum(chi, red);
        if (threadIdx.x == 0) st.chi_part[t] = chi;
    }
}

typedef void (*PGramFn)(DdArgs, DdState, const int32_t*, const int32_t*);
PGramFn pick_gram(int nt) {
    return nt == 1 ? ddp_gram_kernel<1> : nt == 2 ? ddp_gram_kernel<2> : ddp_gram_kernel<3>;
}
typedef void (*PGramRFn)(DdArgs, DdState);
PGramRFn pick_gram_r(int nt) {
    return nt == 1 ? ddp_gram_r_kernel<1> : nt == 2 ? ddp_gram_r_kernel<2> : ddp_gram_r_kernel<3>;
}

void launch_pres_tiles(const wcal_plan* plan, const DdArgs& a, const DdState& st, hipStream_t s, int slot) {
    const size_t sm = pg_bytes(a.n_dir, a.n_ant);
    const int g = dd_grid(plan, reinterpret_cast<const void*>(ddp_resid_kernel), sm, st.ntiles);
    prof_begin(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(ddp_resid_kernel, dim3(g), dim3(DT), sm, s, a, st, slot);
    prof_end(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(dd_chi2_kernel, dim3((a.n_int + DT - 1) / DT), dim3(DT), 0, s, a, st);
}

}  // namespace

size_t ddp_stats_bytes(const wcal_problem& p) { return dd_state_bytes(p, prec_floats(p.n_dir)); }
size_t ddp_lds_need(int nd, int na) {
    const size_t ant = pant_smem(nd, na), g = pg_bytes(nd, na);
    size_t need = ant + std::max(kernel_static_lds(reinterpret_cast<const void*>(ddp_ant_kernel<false>)),
                                 kernel_static_lds(reinterpret_cast<const void*>(ddp_ant_kernel<true>)));
    need = std::max(need, g + kernel_static_lds(reinterpret_cast<const void*>(ddp_resid_kernel)));
    return std::max(need, g + kernel_static_lds(reinterpret_cast<const void*>(pick_gram_r(ptiles(nd, true)))));
}
int ddp_max_dir() { return PND; }
const char* ddp_pass_kernel_name(int nd) {
    const int nt = ptiles(nd, false);
    return nt == 1 ? "ddp_gram_kernel<1>" : nt == 2 ? "ddp_gram_kernel<2>" : "ddp_gram_kernel<3>";
}

hipError_t launch_ddp_solve(const wcal_plan* plan, const DdArgs& a0, hipStream_t s) {
    DdArgs a = a0;
    const int nd = a.n_dir, na = a.n_ant;
    DdState st = dd_state_of(plan, prec_floats(nd));
    const int nctr = 2 * (a.max_iter + 2) + 4;
    const int64_t nblk = (int64_t)a.n_int * ((a.n_bl + PGB - 1) / PGB);
    const PGramFn gram = pick_gram(ptiles(nd, false));
    const int gg = dd_grid(plan, reinterpret_cast<const void*>(gram), 0, nblk);
    const size_t asm_ = pant_smem(nd, na);
    prof_begin(plan, WCAL_K_OTHER, s);
    hipLaunchKernelGGL(dd_init_kernel, dim3((std::max(a.n_int, nctr) + DT - 1) / DT), dim3(DT), 0, s, a, st, 1, nctr);
    prof_end(plan, WCAL_K_OTHER, s);
    const bool stats = plan->prob.mode == WCAL_MODE_STATS;
    if (stats) {
        prof_begin(plan, WCAL_K_STATS, s);
        hipLaunchKernelGGL(gram, dim3(gg), dim3(DT), 0, s, a, st, (const int32_t*)nullptr, (const int32_t*)nullptr);
        prof_end(plan, WCAL_K_STATS, s);
    }
    for (int it = 0; it < a.max_iter; ++it) {
        DdState sti = st;
        sti.ctr = st.ctr + dd_pop_slot(it);      // Gram pops of this update at sti.ctr[0]
        if (!stats) {
            const int32_t* lst = it == 0 ? nullptr : st.alist + (it & 1) * a.n_int;
            prof_begin(plan, WCAL_K_PASS, s);
            const int32_t* nl = st.ctr + dd_nlist_slot(it);
            hipLaunchKernelGGL(gram, dim3(gg), dim3(DT), 0, s, a, sti, lst, nl);
            prof_end(plan, WCAL_K_PASS, s);
        }
        prof_begin(plan, stats ? WCAL_K_SOLVE_STATS : WCAL_K_UPDATE, s);
        hipLaunchKernelGGL(ddp_ant_kernel<false>, dim3(a.n_int * na), dim3(DT), asm_, s, a, st, it);
        hipLaunchKernelGGL(dd_finish_kernel, dim3(a.n_int), dim3(DT), 0, s, a, st, it);
        prof_end(plan, stats ? WCAL_K_SOLVE_STATS : WCAL_K_UPDATE, s);
        if (watch_stop(plan, s, st.ctr + dd_nlist_slot(it + 1), it)) break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.residual || a.chi2) {
        a.gains_in = a.gains;
        launch_pres_tiles(plan, a, st, s, nctr - 1);
    }
    return hipGetLastError();
}

hipError_t launch_ddp_accumulate(const wcal_plan* plan, const DdArgs& a, hipStream_t s) {
    const int nd = a.n_dir, na = a.n_ant;
    DdState st = dd_state_of(plan, prec_floats(nd));
    hipLaunchKernelGGL(dd_init_kernel, dim3(1), dim3(DT), 0, s, a, st, 0, 4);
    const int64_t nblk = (int64_t)a.n_int * ((a.n_bl + PGB - 1) / PGB);
    const PGramRFn gram = pick_gram_r(ptiles(nd, true));
    const size_t gsm = pg_bytes(nd, na);
    const int gg = dd_grid(plan, reinterpret_cast<const void*>(gram), gsm, nblk);
    hipLaunchKernelGGL(gram, dim3(gg), dim3(DT), gsm, s, a, st);
    hipLaunchKernelGGL(ddp_ant_kernel<true>, dim3(a.n_int * na), dim3(DT), pant_smem(nd, na), s, a, st, 0);
    hipLaunchKernelGGL(ddp_chi2_bl_kernel, dim3((a.n_int + DT - 1) / DT), dim3(DT), 0, s, a, st);
    return hipGetLastError();
}

hipError_t launch_ddp_residual(const wcal_plan* plan, const DdArgs& a, hipStream_t s) {
    DdState st = dd_state_of(plan, prec_floats(a.n_dir));
    hipLaunchKernelGGL(dd_init_kernel, dim3(1), dim3(DT), 0, s, a, st, 0, 4);
    launch_pres_tiles(plan, a, st, s, 3);
    return hipGetLastError();
}
