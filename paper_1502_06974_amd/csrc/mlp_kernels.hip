// Warm-start network on gfx950: a three-layer perceptron (tanh hidden layers, linear
// output, optionally plus the input: a skip connection) with hand-written FP32 kernels
// for the forward pass, backpropagation of the mean-squared error and Adam (Kingma & Ba
// 2015).  Parameters live flat in device memory
// in the order W1 [d_in][d_h], b1, W2 [d_h][d_h], b2, W3 [d_h][d_out], b3; rows of x and y
// are samples.  Initial parameters are supplied by the caller.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "wcal_internal.h"

struct wcal_mlp {
    int device = 0;
    int d_in = 0, d_h = 0, d_out = 0, max_batch = 0;
    bool skip = false;         // y += x (d_in == d_out)
    int64_t np = 0;
    int64_t step = 0;
    float* params = nullptr;   // [np]
    float* grads = nullptr;    // [np]
    float* m = nullptr;        // Adam first moment
    float* v = nullptr;        // Adam second moment
    float* h1 = nullptr;       // [max_batch][d_h]
    float* h2 = nullptr;       // [max_batch][d_h]
    float* y = nullptr;        // [max_batch][d_out]
    float* dy = nullptr;       // [max_batch][d_out]
    float* d2 = nullptr;       // [max_batch][d_h]
    float* d1 = nullptr;       // [max_batch][d_h]
    double* loss = nullptr;    // [1]
};

namespace {

constexpr int BT = 64;    // output tile
constexpr int BK = 16;    // depth of one LDS stage

enum Epi { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_TANH_BACK = 3, EPI_BIAS_SKIP = 4 };

// C[M][N] = op(A)[M][K] op(B)[K][N], then the epilogue:
//   EPI_BIAS       C += bias[n]
//   EPI_BIAS_TANH  C = tanh(C + bias[n])
//   EPI_TANH_BACK  C *= 1 - aux[m][n]^2   (gradient through a tanh whose output is aux)
//   EPI_BIAS_SKIP  C += bias[n] + aux[m][n] (skip connection, aux = the input rows)
// op(A) = A stored [M][K] (TA = false) or [K][M] (TA = true); op(B) = B stored [K][N]
// (TB = false) or [N][K] (TB = true).  256 threads, 4 x 4 outputs each, 64 x 64 tile.
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(int M, int N, int K, const float* __restrict__ A,
                                                   const float* __restrict__ B, float* __restrict__ C,
                                                   const float* __restrict__ bias, const float* __restrict__ aux) {
    __shared__ float As[BK][BT + 1];
    __shared__ float Bs[BK][BT + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += BK) {
        // stage A tile: As[kk][mm] = op(A)[m0 + mm][k0 + kk]
        for (int i = threadIdx.x; i < BK * BT; i += blockDim.x) {
            const int kk = i / BT, mm = i % BT;
            const int gm = m0 + mm, gk = k0 + kk;
            float val = 0.f;
            if (gm < M && gk < K) val = TA ? A[(int64_t)gk * M + gm] : A[(int64_t)gm * K + gk];
            As[kk][mm] = val;
        }
        for (int i = threadIdx.x; i < BK * BT; i += blockDim.x) {
            const int kk = i / BT, nn = i % BT;
            const int gn = n0 + nn, gk = k0 + kk;
            float val = 0.f;
            if (gn < N && gk < K) val = TB ? B[(int64_t)gn * K + gk] : B[(int64_t)gk * N + gn];
            Bs[kk][nn] = val;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + ty + 16 * i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx + 16 * j;
            if (gn >= N) continue;
            float c = acc[i][j];
            if (EPI == EPI_BIAS) c += bias[gn];
            if (EPI == EPI_BIAS_SKIP) c += bias[gn] + aux[(int64_t)gm * N + gn];
            if (EPI == EPI_BIAS_TANH) c = tanhf(c + bias[gn]);
            if (EPI == EPI_TANH_BACK) {
                const float h = aux[(int64_t)gm * N + gn];
                c *= 1.f - h * h;
            }
            C[(int64_t)gm * N + gn] = c;
        }
    }
}

// out[n] = sum over rows m of X[m][n] (bias gradients), one thread per column
__global__ void colsum_kernel(int M, int N, const float* __restrict__ X, float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += X[(int64_t)m * N + n];
    out[n] = s;
}

// dy = 2 (y - t) / (M N); loss = mean (y - t)^2 (FP64, one workgroup)
__global__ void __launch_bounds__(256) mse_kernel(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                                                  float* __restrict__ dy, double* loss) {
    __shared__ double red[256];
    double s = 0.0;
    const float sc = 2.f / (float)n;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float e = y[i] - t[i];
        dy[i] = sc * e;
        s += (double)e * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (double)n;
}

__global__ void zero_kernel(int64_t n, float* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

template <bool TA, bool TB, int EPI>
void gemm(int M, int N, int K, const float* A, const float* B, float* C, const float* bias, const float* aux,
          hipStream_t s) {
    dim3 grid((N + BT - 1) / BT, (M + BT - 1) / BT);
    hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, A, B, C, bias, aux);
}

struct Views {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
};

Views views(const wcal_mlp* n) {
    Views v;
    const float* p = n->params;
    float* g = n->grads;
    const int64_t s1 = (int64_t)n->d_in * n->d_h, s2 = n->d_h, s3 = (int64_t)n->d_h * n->d_h, s4 = n->d_h,
                  s5 = (int64_t)n->d_h * n->d_out;
    v.W1 = p; v.b1 = p + s1; v.W2 = v.b1 + s2; v.b2 = v.W2 + s3; v.W3 = v.b2 + s4; v.b3 = v.W3 + s5;
    v.gW1 = g; v.gb1 = g + s1; v.gW2 = v.gb1 + s2; v.gb2 = v.gW2 + s3; v.gW3 = v.gb2 + s4; v.gb3 = v.gW3 + s5;
    return v;
}

void forward(const wcal_mlp* n, const float* x, int B, float* y, hipStream_t s) {
    const Views v = views(n);
    gemm<false, false, EPI_BIAS_TANH>(B, n->d_h, n->d_in, x, v.W1, n->h1, v.b1, nullptr, s);
    gemm<false, false, EPI_BIAS_TANH>(B, n->d_h, n->d_h, n->h1, v.W2, n->h2, v.b2, nullptr, s);
    if (n->skip)
        gemm<false, false, EPI_BIAS_SKIP>(B, n->d_out, n->d_h, n->h2, v.W3, y, v.b3, x, s);
    else
        gemm<false, false, EPI_BIAS>(B, n->d_out, n->d_h, n->h2, v.W3, y, v.b3, nullptr, s);
}

// forward + backward: gradients into n->grads, loss into n->loss
void backward(const wcal_mlp* n, const float* x, const float* t, int B, hipStream_t s) {
    const Views v = views(n);
    forward(n, x, B, n->y, s);
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, s, (int64_t)B * n->d_out, n->y, t, n->dy, n->loss);
    gemm<true, false, EPI_NONE>(n->d_h, n->d_out, B, n->h2, n->dy, v.gW3, nullptr, nullptr, s);
    hipLaunchKernelGGL(colsum_kernel, dim3((n->d_out + 255) / 256), dim3(256), 0, s, B, n->d_out, n->dy, v.gb3);
    gemm<false, true, EPI_TANH_BACK>(B, n->d_h, n->d_out, n->dy, v.W3, n->d2, nullptr, n->h2, s);
    gemm<true, false, EPI_NONE>(n->d_h, n->d_h, B, n->h1, n->d2, v.gW2, nullptr, nullptr, s);
    hipLaunchKernelGGL(colsum_kernel, dim3((n->d_h + 255) / 256), dim3(256), 0, s, B, n->d_h, n->d2, v.gb2);
    gemm<false, true, EPI_TANH_BACK>(B, n->d_h, n->d_h, n->d2, v.W2, n->d1, nullptr, n->h1, s);
    gemm<true, false, EPI_NONE>(n->d_in, n->d_h, B, x, n->d1, v.gW1, nullptr, nullptr, s);
    hipLaunchKernelGGL(colsum_kernel, dim3((n->d_h + 255) / 256), dim3(256), 0, s, B, n->d_h, n->d1, v.gb1);
}

int mfail(int code, const char* msg) { return wcal_error(code, msg); }
int mfail(int code, const std::string& msg) { return wcal_error(code, msg); }

// Weight file: one line of JSON naming the network, then the parameters, the Adam first and
// second moments, each n_params little-endian float32 values.
const char* kMlpFormat = "wcal-mlp";
constexpr int kMlpVersion = 1;

bool little_endian() {
    const uint16_t one = 1;
    unsigned char b;
    std::memcpy(&b, &one, 1);
    return b == 1;
}

// Integer value of "key": N in a flat JSON object, or false when absent.
bool json_int(const std::string& h, const char* key, int64_t& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t i = h.find(k);
    if (i == std::string::npos) return false;
    i = h.find(':', i + k.size());
    if (i == std::string::npos) return false;
    const char* c = h.c_str() + i + 1;
    char* end = nullptr;
    const long long v = std::strtoll(c, &end, 10);
    if (end == c) return false;
    out = v;
    return true;
}

// String value of "key": "value", or false when absent.
bool json_str(const std::string& h, const char* key, std::string& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t i = h.find(k);
    if (i == std::string::npos) return false;
    i = h.find(':', i + k.size());
    if (i == std::string::npos) return false;
    const size_t a = h.find('"', i + 1);
    if (a == std::string::npos) return false;
    const size_t b = h.find('"', a + 1);
    if (b == std::string::npos) return false;
    out = h.substr(a + 1, b - a - 1);
    return true;
}

}  // namespace

extern "C" {

int wcal_mlp_create(int32_t d_in, int32_t d_hidden, int32_t d_out, int32_t max_batch, int32_t skip, int device,
                    wcal_mlp** out) {
    if (!out) return mfail(WCAL_EINVAL, "out is NULL");
    *out = nullptr;
    if (d_in < 1 || d_hidden < 1 || d_out < 1 || max_batch < 1) return mfail(WCAL_EINVAL, "sizes must be >= 1");
    if (skip && d_in != d_out) return mfail(WCAL_EINVAL, "a skip connection needs d_in == d_out");
    if ((int64_t)d_in * d_hidden > (1 << 26) || (int64_t)max_batch * d_hidden > (1 << 28))
        return mfail(WCAL_ESHAPE, "network too large");
    if (hipSetDevice(device) != hipSuccess) return mfail(WCAL_EHIP, "hipSetDevice failed");
    auto* n = new wcal_mlp();
    n->device = device;
    n->d_in = d_in; n->d_h = d_hidden; n->d_out = d_out; n->max_batch = max_batch;
    n->skip = skip != 0;
    n->np = (int64_t)d_in * d_hidden + d_hidden + (int64_t)d_hidden * d_hidden + d_hidden +
            (int64_t)d_hidden * d_out + d_out;
    float** bufs[] = {&n->params, &n->grads, &n->m, &n->v};
    for (float** b : bufs)
        if (hipMalloc(reinterpret_cast<void**>(b), n->np * sizeof(float)) != hipSuccess) {
            wcal_mlp_destroy(n);
            return mfail(WCAL_ENOMEM, "parameter allocation failed");
        }
    const int64_t bh = (int64_t)max_batch * d_hidden, bo = (int64_t)max_batch * d_out;
    if (hipMalloc(reinterpret_cast<void**>(&n->h1), bh * sizeof(float)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&n->h2), bh * sizeof(float)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&n->d1), bh * sizeof(float)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&n->d2), bh * sizeof(float)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&n->y), bo * sizeof(float)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&n->dy), bo * sizeof(float)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&n->loss), sizeof(double)) != hipSuccess) {
        wcal_mlp_destroy(n);
        return mfail(WCAL_ENOMEM, "workspace allocation failed");
    }
    if (hipMemset(n->m, 0, n->np * sizeof(float)) != hipSuccess ||
        hipMemset(n->v, 0, n->np * sizeof(float)) != hipSuccess ||
        hipMemset(n->params, 0, n->np * sizeof(float)) != hipSuccess) {
        wcal_mlp_destroy(n);
        return mfail(WCAL_EHIP, "hipMemset failed");
    }
    *out = n;
    return WCAL_OK;
}

void wcal_mlp_destroy(wcal_mlp* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    for (void* p : {(void*)n->params, (void*)n->grads, (void*)n->m, (void*)n->v, (void*)n->h1, (void*)n->h2,
                    (void*)n->y, (void*)n->dy, (void*)n->d2, (void*)n->d1, (void*)n->loss})
        if (p) (void)hipFree(p);
    delete n;
}

int64_t wcal_mlp_num_params(const wcal_mlp* n) { return n ? n->np : -1; }

int wcal_mlp_set_params(wcal_mlp* n, const float* params, void* stream) {
    if (!n || !params) return mfail(WCAL_EINVAL, "NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(n->params, params, n->np * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return mfail(WCAL_EHIP, "copy failed");
    // Adam moments restart with the new parameters (a fill kernel, not a memset node)
    const unsigned g = (unsigned)((n->np + 255) / 256);
    hipLaunchKernelGGL(zero_kernel, dim3(g), dim3(256), 0, s, n->np, n->m);
    hipLaunchKernelGGL(zero_kernel, dim3(g), dim3(256), 0, s, n->np, n->v);
    n->step = 0;
    return WCAL_OK;
}

int wcal_mlp_get_params(const wcal_mlp* n, float* params, void* stream) {
    if (!n || !params) return mfail(WCAL_EINVAL, "NULL argument");
    if (hipMemcpyAsync(params, n->params, n->np * sizeof(float), hipMemcpyDeviceToDevice,
                       reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
        return mfail(WCAL_EHIP, "copy failed");
    return WCAL_OK;
}

int wcal_mlp_save(const wcal_mlp* n, const char* path) {
    if (!n || !path) return mfail(WCAL_EINVAL, "NULL argument");
    if (!little_endian()) return mfail(WCAL_EIO, "weight files are little-endian; this host is not");
    if (hipSetDevice(n->device) != hipSuccess) return mfail(WCAL_EHIP, "hipSetDevice failed");
    std::vector<float> host(3 * (size_t)n->np);
    const float* src[3] = {n->params, n->m, n->v};
    for (int i = 0; i < 3; ++i)
        if (hipMemcpy(host.data() + i * (size_t)n->np, src[i], n->np * sizeof(float), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return mfail(WCAL_EHIP, "reading the parameters failed");
    char head[512];
    std::snprintf(head, sizeof(head),
                  "{\"format\": \"%s\", \"version\": %d, \"d_in\": %d, \"d_hidden\": %d, \"d_out\": %d, "
                  "\"skip\": %d, \"n_params\": %lld, \"adam_step\": %lld, \"dtype\": \"float32\", "
                  "\"byteorder\": \"little\", \"sections\": [\"params\", \"adam_m\", \"adam_v\"]}\n",
                  kMlpFormat, kMlpVersion, n->d_in, n->d_h, n->d_out, n->skip ? 1 : 0, (long long)n->np,
                  (long long)n->step);
    FILE* f = std::fopen(path, "wb");
    if (!f) return mfail(WCAL_EIO, std::string("cannot open ") + path + " for writing");
    const size_t len = std::strlen(head);
    const bool ok = std::fwrite(head, 1, len, f) == len &&
                    std::fwrite(host.data(), sizeof(float), host.size(), f) == host.size();
    if (std::fclose(f) != 0 || !ok) return mfail(WCAL_EIO, std::string("writing ") + path + " failed");
    return WCAL_OK;
}

int wcal_mlp_load(wcal_mlp* n, const char* path) {
    if (!n || !path) return mfail(WCAL_EINVAL, "NULL argument");
    if (!little_endian()) return mfail(WCAL_EIO, "weight files are little-endian; this host is not");
    FILE* f = std::fopen(path, "rb");
    if (!f) return mfail(WCAL_EIO, std::string("cannot open ") + path);
    std::string head;
    for (int c; (c = std::fgetc(f)) != EOF && c != '\n';) {
        head.push_back((char)c);
        if (head.size() > 4096) break;
    }
    std::string fmt, dtype, order;
    int64_t ver = 0, di = 0, dh = 0, dout = 0, skip = 0, np = 0, step = 0;
    if (!json_str(head, "format", fmt) || fmt != kMlpFormat || !json_int(head, "version", ver) ||
        ver != kMlpVersion || !json_int(head, "d_in", di) || !json_int(head, "d_hidden", dh) ||
        !json_int(head, "d_out", dout) || !json_int(head, "skip", skip) || !json_int(head, "n_params", np) ||
        !json_int(head, "adam_step", step) || !json_str(head, "dtype", dtype) || dtype != "float32" ||
        !json_str(head, "byteorder", order) || order != "little") {
        std::fclose(f);
        return mfail(WCAL_EIO, std::string(path) + " is not a weight file of this library (bad header)");
    }
    if (di != n->d_in || dh != n->d_h || dout != n->d_out || (skip != 0) != n->skip || np != n->np) {
        std::fclose(f);
        return mfail(WCAL_EINVAL, std::string(path) + " holds a network of another shape");
    }
    std::vector<float> host(3 * (size_t)n->np);
    const bool ok = std::fread(host.data(), sizeof(float), host.size(), f) == host.size();
    std::fclose(f);
    if (!ok) return mfail(WCAL_EIO, std::string(path) + " is truncated");
    if (hipSetDevice(n->device) != hipSuccess) return mfail(WCAL_EHIP, "hipSetDevice failed");
    float* dst[3] = {n->params, n->m, n->v};
    for (int i = 0; i < 3; ++i)
        if (hipMemcpy(dst[i], host.data() + i * (size_t)n->np, n->np * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess)
            return mfail(WCAL_EHIP, "writing the parameters failed");
    n->step = step;
    return WCAL_OK;
}

int wcal_mlp_forward(wcal_mlp* n, const float* x, int32_t batch, float* y, void* stream) {
    if (!n || !x || !y) return mfail(WCAL_EINVAL, "NULL argument");
    if (batch < 1 || batch > n->max_batch) return mfail(WCAL_ESHAPE, "batch outside [1, max_batch]");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    forward(n, x, batch, y, s);
    return hipGetLastError() == hipSuccess ? WCAL_OK : mfail(WCAL_EHIP, "launch failed");
}

int wcal_mlp_gradients(wcal_mlp* n, const float* x, const float* t, int32_t batch, float* grads, double* loss,
                       void* stream) {
    if (!n || !x || !t) return mfail(WCAL_EINVAL, "NULL argument");
    if (batch < 1 || batch > n->max_batch) return mfail(WCAL_ESHAPE, "batch outside [1, max_batch]");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    backward(n, x, t, batch, s);
    if (grads && hipMemcpyAsync(grads, n->grads, n->np * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return mfail(WCAL_EHIP, "copy failed");
    if (loss && hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return mfail(WCAL_EHIP, "copy failed");
    return hipGetLastError() == hipSuccess ? WCAL_OK : mfail(WCAL_EHIP, "launch failed");
}

int wcal_mlp_train_step(wcal_mlp* n, const float* x, const float* t, int32_t batch, float lr, double* loss,
                        void* stream) {
    if (!n || !x || !t) return mfail(WCAL_EINVAL, "NULL argument");
    if (batch < 1 || batch > n->max_batch) return mfail(WCAL_ESHAPE, "batch outside [1, max_batch]");
    if (!(lr > 0.f)) return mfail(WCAL_EINVAL, "lr must be > 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    backward(n, x, t, batch, s);
    n->step += 1;
    const float c1 = 1.f - powf(0.9f, (float)n->step), c2 = 1.f - powf(0.999f, (float)n->step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n->np + 255) / 256)), dim3(256), 0, s, n->np, n->params,
                       n->grads, n->m, n->v, lr, c1, c2);
    if (loss && hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return mfail(WCAL_EHIP, "copy failed");
    return hipGetLastError() == hipSuccess ? WCAL_OK : mfail(WCAL_EHIP, "launch failed");
}

}  // extern "C"
