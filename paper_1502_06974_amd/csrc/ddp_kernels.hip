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
// T = Ar^T Ai, Im = T - T^T), an off-diagonal tile pair four (Re as before,
// Im = Ar^T Bi - Ai^T Br).  Flagged samples enter as zeros (selected, not multiplied).
// The accumulate pass adds four residual columns vec R, R = D - sum_d G^d_p M^d G^{dH}_q
// formed per sample in the pass, whose products with the model columns give J^H r.
#include "dd_common.h"

using namespace wcal_dev;

namespace {

constexpr int PND = 10;   // directions: 4 (Nd + 2) columns fit three 16-wide tiles
constexpr int PGB = 8;    // baselines per workgroup task (two per wavefront)
constexpr int PGS = 8;    // samples per chunk

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
// LDS bytes of the gains [nd][na][4], rounded up to 16
__host__ __device__ inline size_t pg_bytes(int nd, int na) { return (size_t)nd * na * 4 * sizeof(float2); }
inline size_t pant_smem(int nd, int na) {
    return pg_bytes(nd, na) + ((size_t)(DT / WAVE) * PNOUT + pn_h(nd) + 4 * pn_n(nd)) * sizeof(double2);
}

// ------------------------------------------------------------------ Gram pass
// A workgroup owns PGB consecutive baselines of one interval and walks its samples in
// chunks of PGS.  For each sample the model rows of the PGB baselines are one contiguous
// segment (PGB * 4 Nd complex) and their data rows another (PGB * 4), so a chunk is read
// as 16-byte pieces with consecutive addresses across the workgroup, staged in registers
// while the previous chunk is consumed, and laid out in LDS as [sample][baseline][column].
// Wavefront w runs the MFMAs of baselines 2w and 2w + 1.
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
    // model (or data) row, and a code (LDS float4 slot | sample << 11 | baseline << 14 |
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
                code[r] = (((sm * PGB + bl) * W16 + c) >> 1) | (sm << 11) | (bl << 14);
            } else {
                const int dq = rem - qm, bl = dq >> 1, c = nm + 2 * (dq & 1);
                goff[r] = sm * nbl * 2 + dq;
                code[r] = (((sm * PGB + bl) * W16 + c) >> 1) | (sm << 11) | (bl << 14) | (1 << 17);
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
                const bool ok = cd >= 0 && s0 + ((cd >> 11) & 7) < ns && b0 + ((cd >> 14) & 7) < nbl;
                stage[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (ok) stage[r] = (cd >> 17) ? load_at(db, goff[r]) : load_at(mb, goff[r]);
            }
            const bool fok = fown && s0 + fs < ns && b0 + fb < nbl;
            fstage = 1;
            if (fok) fstage = has_flags ? (uint8_t)(a.flags[row0 + (int64_t)fs * nbl + fb] != 0) : (uint8_t)0;
        };
        floatx4 dre[2][NT], dti[2][NT], ore[2][NT * (NT - 1) / 2 + 1], oim[2][NT * (NT - 1) / 2 + 1];
        int cnt[2] = {0, 0};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int t = 0; t < NT; ++t) { dre[j][t] = floatx4{0.f, 0.f, 0.f, 0.f}; dti[j][t] = dre[j][t]; }
#pragma unroll
            for (int t = 0; t < NT * (NT - 1) / 2 + 1; ++t) { ore[j][t] = floatx4{0.f, 0.f, 0.f, 0.f}; oim[j][t] = ore[j][t]; }
        }
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
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int bl = 2 * w + j;
#pragma unroll
                for (int g = 0; g < PGS / 4; ++g) {
                    const int sl = 4 * g + kk;
                    const bool use = !fbuf[sl][bl];
                    float2 v[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int cc = 16 * t + col;
                        v[t] = (use && cc < nct) ? abuf[sl][bl][cc] : make_float2(0.f, 0.f);
                    }
                    if (use && col == 0) ++cnt[j];
                    int o = 0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        dre[j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[t].x, v[t].x, dre[j][t], 0, 0, 0);
                        dre[j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[t].y, v[t].y, dre[j][t], 0, 0, 0);
                        dti[j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[t].x, v[t].y, dti[j][t], 0, 0, 0);
#pragma unroll
                        for (int u = t + 1; u < NT; ++u, ++o) {
                            ore[j][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[t].x, v[u].x, ore[j][o], 0, 0, 0);
                            ore[j][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[t].y, v[u].y, ore[j][o], 0, 0, 0);
                            oim[j][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[t].x, v[u].y, oim[j][o], 0, 0, 0);
                            oim[j][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(-v[t].y, v[u].x, oim[j][o], 0, 0, 0);
                        }
                    }
                }
            }
        }
        // epilogue: records of the wavefront's two baselines; the diagonal tiles go through
        // the wavefront's own 2 x 256 floats of the (now free) staging buffer
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
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int b = b0 + 2 * w + j;
            int cj = cnt[j];
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) cj += __shfl_xor(cj, o, WAVE);
            float* rec = st.rec + ((int64_t)k * nbl + b) * RS;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * (lane >> 4) + r;
                    tile[i * 16 + col] = dre[j][t][r];
                    tile[256 + i * 16 + col] = dti[j][t][r];
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
                            if (c2 < nct) put(rec, c1, c2, ore[j][o][r], oim[j][o][r]);
                        }
                if (lane == 0) reinterpret_cast<int*>(rec)[prec_cnt(nd)] = cj;
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
__global__ void __launch_bounds__(DT) ddp_gram_kernel(DdArgs a, DdState st, const int32_t* list,
                                                      const int32_t* n_list) {
    ddp_gram_body<NT, false>(a, st, list, n_list);
}

template <int NT>
__global__ void __launch_bounds__(DT) ddp_gram_r_kernel(DdArgs a, DdState st) {
    ddp_gram_body<NT, true>(a, st, nullptr, nullptr);
}

// ------------------------------------------------------------------ per-antenna update
// Gram entry (x, y) of a record, any x, y < 4 Nd + 4
__device__ __forceinline__ double2 gram_at(const float* rec, int x, int y, int ncs) {
    if (x <= y) {
        const float* v = rec + 2 * tri(x, y, ncs);
        return make_double2(v[0], v[1]);
    }
    const float* v = rec + 2 * tri(y, x, ncs);
    return make_double2(v[0], -v[1]);
}

__device__ __forceinline__ double2 dcmulc(double2 a, double2 b) {   // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 d2(float2 a) { return make_double2(a.x, a.y); }

// H[i][j] of a packed upper triangle (any i, j)
__device__ __forceinline__ double2 phget(const double2* h, int i, int j, int n) {
    return i <= j ? h[tri(i, j, n)] : dconj(h[tri(j, i, n)]);
}

// In-place Cholesky H = R^H R of the packed upper triangle; false when a pivot <= EPS * H_jj.
__device__ bool pchol_factor(double2* h, int n) {
    for (int i = 0; i < n; ++i) {
        const double hii = h[tri(i, i, n)].x;
        double piv = hii;
        for (int k = 0; k < i; ++k) {
            const double2 r = h[tri(k, i, n)];
            piv -= r.x * r.x + r.y * r.y;
        }
        if (!(piv > WCAL_EPS_PIVOT * hii) || !isfinite(piv)) return false;
        const double rii = sqrt(piv);
        h[tri(i, i, n)] = make_double2(rii, 0.0);
        for (int j = i + 1; j < n; ++j) {
            double2 v = h[tri(i, j, n)];
            for (int k = 0; k < i; ++k) {
                const double2 p = dcmulc(h[tri(k, i, n)], h[tri(k, j, n)]);
                v.x -= p.x; v.y -= p.y;
            }
            h[tri(i, j, n)] = make_double2(v.x / rii, v.y / rii);
        }
    }
    return true;
}

// x = H^-1 c with the factor R of pchol_factor: R^H z = c, then R x = z (x may alias c)
__device__ void pchol_subst(const double2* h, const double2* c, double2* x, int n) {
    for (int i = 0; i < n; ++i) {
        double2 v = c[i];
        for (int k = 0; k < i; ++k) {
            const double2 p = dcmulc(h[tri(k, i, n)], x[k]);
            v.x -= p.x; v.y -= p.y;
        }
        const double rii = h[tri(i, i, n)].x;
        x[i] = make_double2(v.x / rii, v.y / rii);
    }
    for (int i = n - 1; i >= 0; --i) {
        double2 v = x[i];
        for (int k = i + 1; k < n; ++k) {
            const double2 p = dmul(h[tri(i, k, n)], x[k]);
            v.x -= p.x; v.y -= p.y;
        }
        const double rii = h[tri(i, i, n)].x;
        x[i] = make_double2(v.x / rii, v.y / rii);
    }
}

// One workgroup per (interval, antenna): lanes run over the outputs (H packed upper, N,
// and J^H r when accumulating); the four wavefronts take every fourth of the antenna's
// baselines (in CSR order) and their FP64 sums are folded in wavefront order.  Solve mode:
// one lane solves (CohJones: Cholesky, two right-hand sides; AllJones: 2x2 per direction,
// residual form), applies the schedule and writes the candidate gains and its share of the
// relative-change norms.  Accumulate mode writes the blocks instead.
template <bool ACC>
__global__ void __launch_bounds__(DT) ddp_ant_kernel(DdArgs a, DdState st, int it) {
    extern __shared__ __align__(16) unsigned char smem[];
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
    const float2* gk = (ACC ? a.gains_in : a.gains) + (int64_t)k * nd * na * 4;
    for (int i = threadIdx.x; i < nd * na * 4; i += DT) G[i] = gk[i];
    __syncthreads();
    const int RS = prec_floats(nd);
    const float* recs = st.rec + (int64_t)k * nbl * RS;
    const int t0 = st.ant_ptr[p], t1 = st.ant_ptr[p + 1];
    for (int e = lane; e < nout; e += WAVE) {
        double2 acc = make_double2(0.0, 0.0);
        if (e < nh) {
            int r1 = 0, rem = e;
            while (rem >= n2 - r1) { rem -= n2 - r1; ++r1; }
            const int r2 = r1 + rem;
            const int c = r1 >> 1, kr = r1 & 1, ee = r2 >> 1, l = r2 & 1;
            for (int t = t0 + w; t < t1; t += nw) {
                const int code = st.ant_bl[t];
                const int b = code >> 1, side = code & 1;
                const int o = side ? a.ant1[b] : a.ant2[b];
                const float* rec = recs + (int64_t)b * RS;
                const float2* gc = G + (c * na + o) * 4;
                const float2* ge = G + (ee * na + o) * 4;
#pragma unroll
                for (int aa = 0; aa < 2; ++aa)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb) {
                        // W^ce[aa][bb] = sum_j conj(G^c_o[j][aa]) G^e_o[j][bb]
                        const double2 w0 = dcmulc(d2(gc[aa]), d2(ge[bb]));
                        const double2 w1 = dcmulc(d2(gc[2 + aa]), d2(ge[2 + bb]));
                        const double2 wv = make_double2(w0.x + w1.x, w0.y + w1.y);
                        const double2 x = side ? gram_at(rec, 4 * c + 2 * aa + kr, 4 * ee + 2 * bb + l, ncs)
                                               : dconj(gram_at(rec, 4 * c + 2 * kr + aa, 4 * ee + 2 * l + bb, ncs));
                        const double2 pr = dmul(wv, x);
                        acc.x += pr.x; acc.y += pr.y;
                    }
            }
        } else {
            const int f = e - nh;
            const bool jr = f >= nn;
            const int idx = jr ? f - nn : f;
            const int i = idx / n2, cc = idx % n2, ee = cc >> 1, l = cc & 1;
            for (int t = t0 + w; t < t1; t += nw) {
                const int code = st.ant_bl[t];
                const int b = code >> 1, side = code & 1;
                const int o = side ? a.ant1[b] : a.ant2[b];
                const float* rec = recs + (int64_t)b * RS;
                const float2* ge = G + (ee * na + o) * 4;
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb) {
                        const int x = side ? 4 * ee + 2 * bb + l : 4 * ee + 2 * l + bb;
                        const int y = side ? 2 * j + i : 2 * i + j;
                        double2 v;
                        if (jr) {
                            const float* q = rec + prec_w(nd) + 2 * (4 * x + y);
                            v = make_double2(q[0], q[1]);
                        } else {
                            v = gram_at(rec, x, nm + y, ncs);
                        }
                        if (side) v = dconj(v);
                        const double2 pr = dmul(d2(ge[2 * j + bb]), v);
                        acc.x += pr.x; acc.y += pr.y;
                    }
            }
        }
        part[w * PNOUT + e] = acc;
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
    if (threadIdx.x == 0) {
        bool fin = true;
        for (int i = 0; i < nh + nn; ++i) fin = fin && isfinite(H[i].x) && isfinite(H[i].y);
        bool ok = true;
        // stacked gains of this antenna: Gs[i][2 d + l] = G^d[i][l]
        auto gs = [&](int i, int cc) { return d2(G[((cc >> 1) * na + p) * 4 + 2 * i + (cc & 1)]); };
        if (a.algo == WCAL_COHJONES) {
            ok = fin && pchol_factor(H, n2);
            if (ok)
                for (int i = 0; i < 2; ++i) {
                    // rows of G H = N: H x = conj(row i of N), row i of G = conj(x)
                    for (int cc = 0; cc < n2; ++cc) X[i * n2 + cc] = dconj(N[i * n2 + cc]);
                    pchol_subst(H, X + i * n2, X + i * n2, n2);
                    for (int cc = 0; cc < n2; ++cc) X[i * n2 + cc] = dconj(X[i * n2 + cc]);
                }
        } else {
            // AllJones: J^H r = N - G H, then G^d + (J^H r)^d (H^dd)^-1 per direction
            for (int i = 0; i < 2; ++i)
                for (int cc = 0; cc < n2; ++cc) {
                    double2 v = N[i * n2 + cc];
                    for (int c2 = 0; c2 < n2; ++c2) {
                        const double2 pr = dmul(gs(i, c2), phget(H, c2, cc, n2));
                        v.x -= pr.x; v.y -= pr.y;
                    }
                    JR[i * n2 + cc] = v;
                }
            for (int d = 0; d < nd; ++d) {
                const double z00 = H[tri(2 * d, 2 * d, n2)].x, z11 = H[tri(2 * d + 1, 2 * d + 1, n2)].x;
                const double2 z01 = H[tri(2 * d, 2 * d + 1, n2)];
                const double det = z00 * z11 - (z01.x * z01.x + z01.y * z01.y);
                const bool sing = !(z00 > 0.0) || !(det > WCAL_EPS_PIVOT * z00 * z11);
                for (int i = 0; i < 2; ++i) {
                    const double2 j0 = JR[i * n2 + 2 * d], j1 = JR[i * n2 + 2 * d + 1];
                    const double2 g0 = gs(i, 2 * d), g1 = gs(i, 2 * d + 1);
                    if (sing || !fin) {
                        X[i * n2 + 2 * d] = g0;
                        X[i * n2 + 2 * d + 1] = g1;
                        continue;
                    }
                    // Z^-1 = [[z11, -z01], [-conj(z01), z00]] / det
                    const double2 a0 = dmul(j1, dconj(z01)), a1 = dmul(j0, z01);
                    X[i * n2 + 2 * d] = make_double2(g0.x + (j0.x * z11 - a0.x) / det, g0.y + (j0.y * z11 - a0.y) / det);
                    X[i * n2 + 2 * d + 1] = make_double2(g1.x + (j1.x * z00 - a1.x) / det,
                                                         g1.y + (j1.y * z00 - a1.y) / det);
                }
                if (sing) ok = false;
            }
        }
        const bool avg = avg_step(it, a.schedule);
        double dsum = 0.0, nsum = 0.0;
        float2* gn = st.gn + (int64_t)k * nd * na * 4;
        for (int d = 0; d < nd; ++d)
            for (int i = 0; i < 2; ++i)
                for (int l = 0; l < 2; ++l) {
                    const double2 go = gs(i, 2 * d + l);
                    double2 v = (a.algo == WCAL_COHJONES && !ok) ? go : X[i * n2 + 2 * d + l];
                    if (avg) v = make_double2(0.5 * (go.x + v.x), 0.5 * (go.y + v.y));
                    const float2 g = make_float2((float)v.x, (float)v.y);
                    gn[(d * na + p) * 4 + 2 * i + l] = g;
                    const double dr = (double)g.x - go.x, di = (double)g.y - go.y;
                    dsum += dr * dr + di * di;
                    nsum += (double)g.x * g.x + (double)g.y * g.y;
                }
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
                    for (int d = 0; d < nd; ++d) {
                        const J2 M = load_j2(a.model, row * nd + d);
                        const float2* gp = gsh + (d * na + p) * 4;
                        const float2* gq = gsh + (d * na + q) * 4;
                        const J2 Gp{gp[0], gp[1], gp[2], gp[3]}, Gq{gq[0], gq[1], gq[2], gq[3]};
                        R = jsub(R, mulH(mul(Gp, M), Gq));
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
size_t ddp_smem_bytes(int nd, int na) { return pant_smem(nd, na); }
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
