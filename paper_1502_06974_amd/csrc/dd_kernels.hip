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
#include "di_common.h"

using namespace wcal_dev;

namespace {

constexpr int DT = 256;          // workgroup size
constexpr int NDMAX = 14;        // Nd + 2 augmented columns fit one 16-wide MFMA tile

typedef float floatx4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline int ntri(int nd) { return nd * (nd + 1) / 2; }
// packed index of (i, j), i <= j < nd, row-major upper triangle
__host__ __device__ inline int tri(int i, int j, int nd) { return i * nd - i * (i - 1) / 2 + (j - i); }
// floats per baseline record: X (upper, complex), Z, W (complex), sum |d|^2, count
__host__ __device__ inline int rec_floats(int nd) {
    const int n = 2 * ntri(nd) + 4 * nd + 2;
    return (n + 3) / 4 * 4;
}
__host__ __device__ inline int rec_z(int nd) { return 2 * ntri(nd); }
__host__ __device__ inline int rec_w(int nd) { return 2 * ntri(nd) + 2 * nd; }
__host__ __device__ inline int rec_d2(int nd) { return 2 * ntri(nd) + 4 * nd; }
__host__ __device__ inline int rec_cnt(int nd) { return 2 * ntri(nd) + 4 * nd + 1; }

struct DdState {
    float* rec;          // [n_int][n_bl][rec_floats]
    double* chi_bl;      // [n_int][n_bl] chi^2 per baseline (accumulate)
    const int32_t* ant_ptr;  // [n_ant + 1] CSR of (baseline, side) per antenna
    const int32_t* ant_bl;   // [2 n_bl]: 2 b + side (side 0: antenna is ant1, 1: ant2)
    int32_t* active;     // [n_int]
    int32_t* ctr;        // work counters
    const Tile* tiles;
    const int32_t* tile_off;
    int32_t ntiles;
    double* chi_part;    // [ntiles]
};

__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

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

// CohJones GN value for one antenna: Cholesky H = R^H R in place (upper packed), then
// R^H z = c, R x = z.  Returns false (gain kept) when a pivot <= EPS * H_jj.
__device__ bool chol_solve(double2* h, const double2* c, double2* x, int nd) {
    for (int i = 0; i < nd; ++i) {
        const double hii = h[tri(i, i, nd)].x;
        double piv = hii;
        for (int k = 0; k < i; ++k) {
            const double2 r = h[tri(k, i, nd)];
            piv -= r.x * r.x + r.y * r.y;
        }
        if (!(piv > WCAL_EPS_PIVOT * hii) || !isfinite(piv)) return false;
        const double rii = sqrt(piv);
        h[tri(i, i, nd)] = make_double2(rii, 0.0);
        for (int j = i + 1; j < nd; ++j) {
            double2 v = h[tri(i, j, nd)];
            for (int k = 0; k < i; ++k) {
                const double2 rki = h[tri(k, i, nd)], rkj = h[tri(k, j, nd)];
                // v -= conj(R[k][i]) R[k][j]
                v.x -= rki.x * rkj.x + rki.y * rkj.y;
                v.y -= rki.x * rkj.y - rki.y * rkj.x;
            }
            h[tri(i, j, nd)] = make_double2(v.x / rii, v.y / rii);
        }
    }
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
    return true;
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

// One update of interval k: per batch of BA antennas form their blocks, solve each
// (CohJones: Cholesky; AllJones: diagonal, residual form), apply the schedule into Gn.
// Then the FP64 relative change decides.  Returns 1 when the interval stops.
__device__ int dd_update_step(const DdArgs& a, const DdState& st, int k, int it, const DdSmem& S, double* red,
                              int* s_flags, uint32_t& status) {
    const int nd = a.n_dir, na = a.n_ant;
    const int nx = ntri(nd);
    if (threadIdx.x == 0) { s_flags[0] = 0; s_flags[1] = 0; }
    const bool avg = avg_step(it, a.schedule);
    double dsum = 0.0, nsum = 0.0;
    for (int p0 = 0; p0 < na; p0 += BA) {
        const int nb = min(BA, na - p0);
        __syncthreads();
        dd_blocks<false>(a, st, k, S.G, p0, nb, S.H, S.C, nullptr, nullptr);
        __syncthreads();
        if (threadIdx.x < nb) {
            const int j = threadIdx.x, p = p0 + j;
            double2* h = S.H + j * nx;
            const double2* c = S.C + j * nd;
            double2* x = S.X + j * NDMAX;
            bool fin = true;
            for (int i = 0; i < nx; ++i) fin = fin && isfinite(h[i].x) && isfinite(h[i].y);
            for (int i = 0; i < nd; ++i) fin = fin && isfinite(c[i].x) && isfinite(c[i].y);
            if (!fin) s_flags[0] = 1;
            bool ok = true;
            if (a.algo == WCAL_COHJONES) {
                ok = fin && chol_solve(h, c, x, nd);
            } else {
                // AllJones: g^d + (c_d - sum_e H[d][e] g^e) / H[d][d], per direction
                for (int d = 0; d < nd; ++d) {
                    const double hdd = hget(h, d, d, nd).x;
                    const float2 gd = S.G[d * na + p];
                    if (!(hdd > 0.0)) {
                        ok = false;
                        x[d] = make_double2(gd.x, gd.y);
                        continue;
                    }
                    double2 jr = c[d];
                    for (int e = 0; e < nd; ++e) {
                        const float2 ge = S.G[e * na + p];
                        const double2 pr = dmul(hget(h, d, e, nd), make_double2(ge.x, ge.y));
                        jr.x -= pr.x; jr.y -= pr.y;
                    }
                    x[d] = make_double2(gd.x + jr.x / hdd, gd.y + jr.y / hdd);
                }
            }
            if (!ok) s_flags[1] = 1;
            for (int d = 0; d < nd; ++d) {
                const float2 go = S.G[d * na + p];
                double nr, ni;
                if (a.algo == WCAL_COHJONES && !ok) { nr = go.x; ni = go.y; }
                else { nr = x[d].x; ni = x[d].y; }
                if (avg) { nr = 0.5 * (go.x + nr); ni = 0.5 * (go.y + ni); }
                const float2 gn = make_float2((float)nr, (float)ni);
                S.Gn[d * na + p] = gn;
                const double dr = (double)gn.x - go.x, di = (double)gn.y - go.y;
                dsum += dr * dr + di * di;
                nsum += (double)gn.x * gn.x + (double)gn.y * gn.y;
            }
        }
    }
    dsum = block_sum(dsum, red);
    nsum = block_sum(nsum, red);
    if (s_flags[0]) { status |= WCAL_NONFINITE; __syncthreads(); return 1; }
    if (s_flags[1]) status |= WCAL_SINGULAR_ANT;
    for (int i = threadIdx.x; i < nd * na; i += blockDim.x) S.G[i] = S.Gn[i];
    __syncthreads();
    const double num = sqrt(dsum), den = sqrt(nsum);
    const double rel = den == 0.0 ? (num == 0.0 ? 0.0 : INFINITY) : num / den;
    if (rel < a.tol) { status |= WCAL_CONVERGED; return 1; }
    return 0;
}

// Iterate updates [it0, it1) of every interval (one workgroup per interval popped from the
// queue).  Per-interval state (status, n_iter, active) lives in global memory so PASS mode
// can call this once per update.
__global__ void __launch_bounds__(DT) dd_iterate_kernel(DdArgs a, DdState st, int it0, int it1) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nd = a.n_dir, na = a.n_ant;
    DdSmem S = dd_smem(smem, nd, na);
    __shared__ double red[DT / WAVE];
    __shared__ int s_flags[2];
    __shared__ int s_k;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_k = atomicAdd(&st.ctr[1], 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_k);
        if (idx >= a.n_int) break;
        const int k = a.order[idx];
        if (!st.active[k]) continue;
        float2* gk = a.gains + (int64_t)k * nd * na;
        for (int i = threadIdx.x; i < nd * na; i += blockDim.x) S.G[i] = gk[i];
        __syncthreads();
        uint32_t status = 0;
        int n_it = a.n_iter[k];
        bool finished = false;
        for (int it = it0; it < it1; ++it) {
            const int stop = dd_update_step(a, st, k, it, S, red, s_flags, status);
            if (status & WCAL_NONFINITE) { finished = true; break; }
            n_it = it + 1;
            if (stop) { finished = true; break; }
        }
        if (!finished && it1 >= a.max_iter) {
            status |= WCAL_MAXITER;
            finished = true;
        }
        for (int i = threadIdx.x; i < nd * na; i += blockDim.x) gk[i] = S.G[i];
        if (threadIdx.x == 0) {
            a.status[k] |= status;
            a.n_iter[k] = n_it;
            if (finished) st.active[k] = 0;
        }
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

__global__ void __launch_bounds__(DT) dd_init_kernel(DdArgs a, DdState st, int init_state, int nctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (init_state && i < a.n_int) {
        a.status[i] = 0;
        a.n_iter[i] = 0;
        st.active[i] = 1;
    }
    if (i < nctr) st.ctr[i] = 0;
}

// Residual rows of one tile: lane <-> baseline, weights g^c_p conj(g^c_q) per round.
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
            float part = 0.f;
            for (int s = T.s0; s < T.s1; ++s) {
                const int64_t row = off + (int64_t)s * nbl + b;
                const bool fl = has_flags && a.flags[row] != 0;
                float2 r = make_float2(0.f, 0.f);
                if (!fl) {
                    r = a.data[row];
                    const float2* m = a.model + row * nd;
#pragma unroll
                    for (int c = 0; c < NDMAX; ++c)
                        if (c < nd) r = csub(r, cmul(w[c], m[c]));
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

__global__ void __launch_bounds__(DT) dd_chi2_kernel(DdArgs a, DdState st) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_int || !a.chi2) return;
    double c = 0.0;
    for (int t = st.tile_off[k]; t < st.tile_off[k + 1]; ++t) c += st.chi_part[t];
    a.chi2[k] = c;
}

int grid_res(const wcal_plan* plan, const void* fn, size_t smem, int64_t work) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, DT, smem) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t g = (int64_t)per_cu * plan->n_cu;
    if (g > work) g = work;
    return (int)(g < 1 ? 1 : g);
}

DdState state_of(const wcal_plan* plan) {
    DdState st;
    const int nd = plan->prob.n_dir;
    st.rec = plan->d_stats;
    st.chi_bl = reinterpret_cast<double*>(plan->d_stats + (size_t)plan->prob.n_int * plan->prob.n_bl * rec_floats(nd));
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

}  // namespace

size_t dd_stats_bytes(const wcal_problem& p) {
    const size_t n = (size_t)p.n_int * p.n_bl;
    return n * rec_floats(p.n_dir) * sizeof(float) + n * sizeof(double);
}

size_t dd_smem_bytes(int nd, int na) { return dd_smem_size(nd, na); }

int dd_max_dir() { return NDMAX; }

static void launch_residual_tiles(const wcal_plan* plan, const DdArgs& a, const DdState& st, hipStream_t s,
                                  int slot) {
    const int g = grid_res(plan, reinterpret_cast<const void*>(dd_resid_kernel), 0, st.ntiles);
    prof_begin(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(dd_resid_kernel, dim3(g), dim3(DT), 0, s, a, st, slot);
    prof_end(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(dd_chi2_kernel, dim3((a.n_int + DT - 1) / DT), dim3(DT), 0, s, a, st);
}

hipError_t launch_dd_solve(const wcal_plan* plan, const DdArgs& a0, hipStream_t s) {
    DdArgs a = a0;
    DdState st = state_of(plan);
    const int nd = a.n_dir, na = a.n_ant;
    const int nctr = 2 * (a.max_iter + 2) + 4;
    const size_t sm = dd_smem_bytes(nd, na);
    const int64_t ntask = (int64_t)a.n_int * a.n_bl;
    const int gg = grid_res(plan, reinterpret_cast<const void*>(dd_gram_kernel<false>), 0, (ntask + 3) / 4);
    const int gi = grid_res(plan, reinterpret_cast<const void*>(dd_iterate_kernel), sm, a.n_int);
    prof_begin(plan, WCAL_K_OTHER, s);
    hipLaunchKernelGGL(dd_init_kernel, dim3((std::max(a.n_int, nctr) + DT - 1) / DT), dim3(DT), 0, s, a, st, 1, nctr);
    prof_end(plan, WCAL_K_OTHER, s);
    if (plan->prob.mode == WCAL_MODE_STATS) {
        prof_begin(plan, WCAL_K_STATS, s);
        hipLaunchKernelGGL(dd_gram_kernel<false>, dim3(gg), dim3(DT), 0, s, a, st, 0);
        prof_end(plan, WCAL_K_STATS, s);
        prof_begin(plan, WCAL_K_SOLVE_STATS, s);
        hipLaunchKernelGGL(dd_iterate_kernel, dim3(gi), dim3(DT), sm, s, a, st, 0, a.max_iter);
        prof_end(plan, WCAL_K_SOLVE_STATS, s);
    } else {
        for (int it = 0; it < a.max_iter; ++it) {
            DdState sti = st;
            sti.ctr = st.ctr + 2 + 2 * it;     // fresh pop counters per update
            prof_begin(plan, WCAL_K_PASS, s);
            hipLaunchKernelGGL(dd_gram_kernel<false>, dim3(gg), dim3(DT), 0, s, a, sti, 1);
            prof_end(plan, WCAL_K_PASS, s);
            prof_begin(plan, WCAL_K_UPDATE, s);
            hipLaunchKernelGGL(dd_iterate_kernel, dim3(gi), dim3(DT), sm, s, a, sti, it, it + 1);
            prof_end(plan, WCAL_K_UPDATE, s);
        }
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
    DdState st = state_of(plan);
    const int nd = a.n_dir, na = a.n_ant;
    const int nctr = 4;
    hipLaunchKernelGGL(dd_init_kernel, dim3(1), dim3(DT), 0, s, a, st, 0, nctr);
    const int64_t ntask = (int64_t)a.n_int * a.n_bl;
    const int gg = grid_res(plan, reinterpret_cast<const void*>(dd_gram_kernel<true>), 0, (ntask + 3) / 4);
    hipLaunchKernelGGL(dd_gram_kernel<true>, dim3(gg), dim3(DT), 0, s, a, st, 0);
    hipLaunchKernelGGL(dd_reduce_kernel, dim3(a.n_int), dim3(DT), dd_smem_bytes(nd, na), s, a, st);
    return hipGetLastError();
}

hipError_t launch_dd_residual(const wcal_plan* plan, const DdArgs& a, hipStream_t s) {
    DdState st = state_of(plan);
    hipLaunchKernelGGL(dd_init_kernel, dim3(1), dim3(DT), 0, s, a, st, 0, 4);
    launch_residual_tiles(plan, a, st, s, 3);
    return hipGetLastError();
}
