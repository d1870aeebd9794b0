// Annealing-schedule network of libshaken: forward, backward and Adam on the
// gfx950 matrix cores (v_mfma_f32_16x16x16_bf16).
//
// 16 -> 128 -> 128 -> 128 -> 16, ReLU on the hidden layers.  Parameters are
// FP32 masters with BF16 copies (round to nearest even); every product takes
// BF16 operands and accumulates in FP32.  Hidden activations and
// back-propagated pre-activation gradients are stored in BF16, the output and
// all parameter gradients in FP32.  Rows are padded to a multiple of 16; padded
// input rows are zero and padded output-gradient rows are zero, so they add
// nothing to the parameter gradients.
#include "shaken.h"
#include "shaken_internal.hpp"

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace shaken {

namespace {

constexpr int NI = SHAKEN_MLP_IN, NH = SHAKEN_MLP_HIDDEN, NO = SHAKEN_MLP_OUT;
constexpr size_t OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH,
                 OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH,
                 OFF_W4 = OFF_B3 + NH, OFF_B4 = OFF_W4 + NO * NH, NPARAM = OFF_B4 + NO;
static_assert(NPARAM == SHAKEN_MLP_NPARAM, "parameter layout");

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

enum Epi { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_MASK = 2, EPI_F32 = 3 };

// C(i, j) = sum_k A(i, k) B(k, j) over one 16 x 16 tile per wave, A(i,k) =
// A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj] (BF16 bits); M, N, K multiples
// of 16.  Lane l holds A(l%16, 4(l/16)+t), B(4(l/16)+t, l%16) and the result
// rows 4(l/16)+t of column l%16, t = 0..3.
template <int EPI>
__global__ __launch_bounds__(64) void k_gemm(int M, int N, int K, const uint16_t *__restrict__ A,
                                             int sai, int sak, const uint16_t *__restrict__ B,
                                             int sbk, int sbj, float *__restrict__ Cf,
                                             uint16_t *__restrict__ Cb, int ldc,
                                             const float *__restrict__ bias,
                                             const uint16_t *__restrict__ mask, int ldm) {
    const int ti = blockIdx.y * 16, tj = blockIdx.x * 16;
    if (ti >= M || tj >= N) return;
    const int l = threadIdx.x;
    const int r16 = l & 15, kq = (l >> 4) * 4;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        v4s a, b;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a[t] = (short)A[(size_t)(ti + r16) * sai + (size_t)(k0 + kq + t) * sak];
            b[t] = (short)B[(size_t)(k0 + kq + t) * sbk + (size_t)(tj + r16) * sbj];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int i = ti + kq + t, j = tj + r16;
        float v = acc[t];
        if (EPI == EPI_HIDDEN) {
            v += bias[j];
            v = v > 0.f ? v : 0.f;
            Cb[(size_t)i * ldc + j] = f2bf(v);
        } else if (EPI == EPI_OUT) {
            Cf[(size_t)i * ldc + j] = v + bias[j];
        } else if (EPI == EPI_MASK) {
            const uint16_t h = mask[(size_t)i * ldm + j];
            v = (h != 0 && !(h & 0x8000u)) ? v : 0.f;  // ReLU derivative from the stored activation
            Cb[(size_t)i * ldc + j] = f2bf(v);
        } else {
            Cf[(size_t)i * ldc + j] = v;
        }
    }
}

// out[j] = sum_i in[i][j] over `rows` rows (BF16 in, FP32 out): one block per column
__global__ __launch_bounds__(256) void k_colsum(const uint16_t *__restrict__ in, int rows, int ld,
                                                float *__restrict__ out) {
    __shared__ float sh[256];
    const int j = blockIdx.x;
    float a = 0.f;
    for (int i = threadIdx.x; i < rows; i += 256) a += bf2f(in[(size_t)i * ld + j]);
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sh[0];
}

// BF16 copy of an FP32 [rows][16] array into [rows_pad][16], zero padding
__global__ void k_rows_to_bf16(const float *__restrict__ in, int rows, int rows_pad,
                               uint16_t *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows_pad * NI) return;
    out[i] = (i / NI) < rows ? f2bf(in[i]) : (uint16_t)0;
}

__global__ void k_params_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ b, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(w[i]);
}

__global__ __launch_bounds__(1024) void k_weight_sum(const float *__restrict__ w, int rows,
                                                     float *__restrict__ out) {
    __shared__ float sh[1024];
    float a = 0.f;
    for (int i = threadIdx.x; i < rows; i += 1024) a += w ? w[i] : 1.f;
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0];
        out[1] = 0.f;  // loss accumulator
    }
}

// dy[r][c] = w_r * 2 (y - target) / W for c < 2, zero elsewhere and on padded
// rows; loss += w_r * sum_c (y - target)^2 / W
__global__ void k_mse_grad(const float *__restrict__ y, const float *__restrict__ tgt,
                           const float *__restrict__ w, int rows, int rows_pad,
                           float *__restrict__ ws, float *__restrict__ dy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows_pad * NO) return;
    const int r = i / NO, c = i % NO;
    float g = 0.f;
    if (r < rows && c < 2) {
        const float wr = (w ? w[r] : 1.f) / ws[0];
        const float d = y[(size_t)r * NO + c] - tgt[(size_t)r * NO + c];
        g = 2.f * wr * d;
        atomicAdd(&ws[1], wr * d * d);
    }
    dy[i] = g;
}

__global__ void k_dy_to_bf16(const float *__restrict__ dy, int rows, int rows_pad,
                             uint16_t *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows_pad * NO) return;
    out[i] = (i / NO) < rows ? f2bf(dy[i]) : (uint16_t)0;
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, uint16_t *__restrict__ wb, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float m = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = m;
    m2[i] = v;
    const float x = w[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    w[i] = x;
    wb[i] = f2bf(x);
}

}  // namespace
}  // namespace shaken

using namespace shaken;

struct shaken_mlp {
    int device = -1;
    hipStream_t stream = nullptr;
    float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    uint16_t *wb = nullptr;
    int cap = 0;       // padded rows of the workspace
    int rows = 0;      // rows of the last forward
    int rows_pad = 0;
    uint16_t *x = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;
    uint16_t *dzo = nullptr, *dza = nullptr, *dzb = nullptr;
    float *yf = nullptr, *dy = nullptr, *ws = nullptr;
};

namespace {

#define MLPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return set_error(e_ == hipErrorOutOfMemory ? SHAKEN_ENOMEM : SHAKEN_EDEVICE,       \
                             (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str());      \
    } while (0)

struct Dev {
    int prev = -1;
    explicit Dev(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (d >= 0 && d != prev) (void)hipSetDevice(d);
    }
    ~Dev() {
        int c = -1;
        if (prev >= 0 && hipGetDevice(&c) == hipSuccess && c != prev) (void)hipSetDevice(prev);
    }
};

template <class T>
void mfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void ws_free(shaken_mlp *m) {
    mfree(m->x);
    mfree(m->h1);
    mfree(m->h2);
    mfree(m->h3);
    mfree(m->dzo);
    mfree(m->dza);
    mfree(m->dzb);
    mfree(m->yf);
    mfree(m->dy);
    m->cap = 0;
}

shaken_status ensure_cap(shaken_mlp *m, int rows_pad) {
    if (rows_pad <= m->cap) return SHAKEN_OK;
    ws_free(m);
    const size_t r = (size_t)rows_pad;
    MLPCHK(hipMalloc((void **)&m->x, r * NI * 2));
    MLPCHK(hipMalloc((void **)&m->h1, r * NH * 2));
    MLPCHK(hipMalloc((void **)&m->h2, r * NH * 2));
    MLPCHK(hipMalloc((void **)&m->h3, r * NH * 2));
    MLPCHK(hipMalloc((void **)&m->dzo, r * NO * 2));
    MLPCHK(hipMalloc((void **)&m->dza, r * NH * 2));
    MLPCHK(hipMalloc((void **)&m->dzb, r * NH * 2));
    MLPCHK(hipMalloc((void **)&m->yf, r * NO * 4));
    MLPCHK(hipMalloc((void **)&m->dy, r * NO * 4));
    m->cap = rows_pad;
    return SHAKEN_OK;
}

template <int EPI>
hipError_t gemm(hipStream_t st, int M, int N, int K, const uint16_t *A, int sai, int sak,
                const uint16_t *B, int sbk, int sbj, float *Cf, uint16_t *Cb, int ldc,
                const float *bias, const uint16_t *mask, int ldm) {
    hipLaunchKernelGGL(k_gemm<EPI>, dim3(N / 16, M / 16), dim3(64), 0, st, M, N, K, A, sai, sak, B,
                       sbk, sbj, Cf, Cb, ldc, bias, mask, ldm);
    return hipGetLastError();
}

int blocks(size_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

extern "C" {

shaken_status shaken_mlp_create(shaken_mlp **out, int32_t device, void *stream) {
    if (!out) return set_error(SHAKEN_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return set_error(SHAKEN_EDEVICE, "no HIP device");
    }
    if (device >= ndev) return set_error(SHAKEN_EINVAL, "device ordinal out of range");
    shaken_mlp *m = new (std::nothrow) shaken_mlp();
    if (!m) return set_error(SHAKEN_ENOMEM, "host allocation failed");
    if (device < 0) (void)hipGetDevice(&device);
    m->device = device;
    m->stream = (hipStream_t)stream;
    Dev guard(device);
    const size_t nb = NPARAM * 4;
    hipError_t e = hipSuccess;
    if ((e = hipMalloc((void **)&m->w, nb)) != hipSuccess || (e = hipMalloc((void **)&m->g, nb)) != hipSuccess ||
        (e = hipMalloc((void **)&m->m1, nb)) != hipSuccess || (e = hipMalloc((void **)&m->m2, nb)) != hipSuccess ||
        (e = hipMalloc((void **)&m->wb, NPARAM * 2)) != hipSuccess || (e = hipMalloc((void **)&m->ws, 16)) != hipSuccess ||
        (e = hipMemsetAsync(m->w, 0, nb, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->g, 0, nb, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->m1, 0, nb, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->m2, 0, nb, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->wb, 0, NPARAM * 2, m->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(m->stream)) != hipSuccess) {
        shaken_mlp_free(m);
        return set_error(e == hipErrorOutOfMemory ? SHAKEN_ENOMEM : SHAKEN_EDEVICE, hipGetErrorString(e));
    }
    *out = m;
    return SHAKEN_OK;
}

shaken_status shaken_mlp_free(shaken_mlp *m) {
    if (!m) return SHAKEN_OK;
    Dev guard(m->device);
    (void)hipStreamSynchronize(m->stream);
    ws_free(m);
    mfree(m->w);
    mfree(m->g);
    mfree(m->m1);
    mfree(m->m2);
    mfree(m->wb);
    mfree(m->ws);
    delete m;
    return SHAKEN_OK;
}

shaken_status shaken_mlp_set_params(shaken_mlp *m, const float *host, size_t n) {
    if (!m || !host || n != NPARAM) return set_error(SHAKEN_EINVAL, "need the network and SHAKEN_MLP_NPARAM values");
    std::vector<float> p(host, host + NPARAM);
    for (float v : p)
        if (!std::isfinite(v)) return set_error(SHAKEN_EINVAL, "parameters must be finite");
    // output rows beyond the two used ones stay zero
    for (size_t i = OFF_W4 + 2 * NH; i < OFF_B4; ++i) p[i] = 0.f;
    for (size_t i = OFF_B4 + 2; i < NPARAM; ++i) p[i] = 0.f;
    Dev guard(m->device);
    MLPCHK(hipMemcpyAsync(m->w, p.data(), NPARAM * 4, hipMemcpyHostToDevice, m->stream));
    MLPCHK(hipMemsetAsync(m->m1, 0, NPARAM * 4, m->stream));
    MLPCHK(hipMemsetAsync(m->m2, 0, NPARAM * 4, m->stream));
    hipLaunchKernelGGL(k_params_to_bf16, dim3(blocks(NPARAM, 256)), dim3(256), 0, m->stream, m->w, m->wb, (int)NPARAM);
    MLPCHK(hipGetLastError());
    MLPCHK(hipStreamSynchronize(m->stream));
    return SHAKEN_OK;
}

shaken_status shaken_mlp_get_params(shaken_mlp *m, float *host, size_t n) {
    if (!m || !host || n != NPARAM) return set_error(SHAKEN_EINVAL, "need the network and SHAKEN_MLP_NPARAM values");
    Dev guard(m->device);
    MLPCHK(hipMemcpyAsync(host, m->w, NPARAM * 4, hipMemcpyDeviceToHost, m->stream));
    MLPCHK(hipStreamSynchronize(m->stream));
    return SHAKEN_OK;
}

shaken_status shaken_mlp_get_grads(shaken_mlp *m, float *host, size_t n) {
    if (!m || !host || n != NPARAM) return set_error(SHAKEN_EINVAL, "need the network and SHAKEN_MLP_NPARAM values");
    Dev guard(m->device);
    MLPCHK(hipMemcpyAsync(host, m->g, NPARAM * 4, hipMemcpyDeviceToHost, m->stream));
    MLPCHK(hipStreamSynchronize(m->stream));
    return SHAKEN_OK;
}

shaken_status shaken_mlp_forward(shaken_mlp *m, const float *x_dev, int32_t batch, float *y_dev) {
    if (!m || !x_dev || !y_dev || batch < 1) return set_error(SHAKEN_EINVAL, "need the network, x, y and batch >= 1");
    Dev guard(m->device);
    const int rp = (batch + 15) / 16 * 16;
    shaken_status st = ensure_cap(m, rp);
    if (st != SHAKEN_OK) return st;
    hipStream_t s = m->stream;
    hipLaunchKernelGGL(k_rows_to_bf16, dim3(blocks((size_t)rp * NI, 256)), dim3(256), 0, s, x_dev, batch, rp, m->x);
    MLPCHK(hipGetLastError());
    const uint16_t *W = m->wb;
    const float *P = m->w;
    // h1 = relu(x W1^T + b1): A(i,k) = x[i][k], B(k,j) = W1[j][k]
    MLPCHK(gemm<EPI_HIDDEN>(s, rp, NH, NI, m->x, NI, 1, W + OFF_W1, 1, NI, nullptr, m->h1, NH, P + OFF_B1, nullptr, 0));
    MLPCHK(gemm<EPI_HIDDEN>(s, rp, NH, NH, m->h1, NH, 1, W + OFF_W2, 1, NH, nullptr, m->h2, NH, P + OFF_B2, nullptr, 0));
    MLPCHK(gemm<EPI_HIDDEN>(s, rp, NH, NH, m->h2, NH, 1, W + OFF_W3, 1, NH, nullptr, m->h3, NH, P + OFF_B3, nullptr, 0));
    MLPCHK(gemm<EPI_OUT>(s, rp, NO, NH, m->h3, NH, 1, W + OFF_W4, 1, NH, m->yf, nullptr, NO, P + OFF_B4, nullptr, 0));
    MLPCHK(hipMemcpyAsync(y_dev, m->yf, (size_t)batch * NO * 4, hipMemcpyDeviceToDevice, s));
    m->rows = batch;
    m->rows_pad = rp;
    return SHAKEN_OK;
}

static shaken_status mlp_backward_from(shaken_mlp *m) {
    // m->dy holds FP32 [rows_pad][16] with zero padded rows
    hipStream_t s = m->stream;
    const int rp = m->rows_pad, rows = m->rows;
    const uint16_t *W = m->wb;
    float *G = m->g;
    hipLaunchKernelGGL(k_dy_to_bf16, dim3(blocks((size_t)rp * NO, 256)), dim3(256), 0, s, m->dy, rows, rp, m->dzo);
    MLPCHK(hipGetLastError());
    // layer 4: dW4 = dz4^T h3 (M=16, N=128, K=rows), db4 = colsum dz4
    MLPCHK(gemm<EPI_F32>(s, NO, NH, rp, m->dzo, 1, NO, m->h3, NH, 1, G + OFF_W4, nullptr, NH, nullptr, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(NO), dim3(256), 0, s, m->dzo, rp, NO, G + OFF_B4);
    MLPCHK(hipGetLastError());
    // dz3 = mask(h3) * (dz4 W4): A(i,k) = dz4[i][k], B(k,j) = W4[k][j]
    MLPCHK(gemm<EPI_MASK>(s, rp, NH, NO, m->dzo, NO, 1, W + OFF_W4, NH, 1, nullptr, m->dza, NH, nullptr, m->h3, NH));
    MLPCHK(gemm<EPI_F32>(s, NH, NH, rp, m->dza, 1, NH, m->h2, NH, 1, G + OFF_W3, nullptr, NH, nullptr, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, m->dza, rp, NH, G + OFF_B3);
    MLPCHK(hipGetLastError());
    MLPCHK(gemm<EPI_MASK>(s, rp, NH, NH, m->dza, NH, 1, W + OFF_W3, NH, 1, nullptr, m->dzb, NH, nullptr, m->h2, NH));
    MLPCHK(gemm<EPI_F32>(s, NH, NH, rp, m->dzb, 1, NH, m->h1, NH, 1, G + OFF_W2, nullptr, NH, nullptr, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, m->dzb, rp, NH, G + OFF_B2);
    MLPCHK(hipGetLastError());
    MLPCHK(gemm<EPI_MASK>(s, rp, NH, NH, m->dzb, NH, 1, W + OFF_W2, NH, 1, nullptr, m->dza, NH, nullptr, m->h1, NH));
    MLPCHK(gemm<EPI_F32>(s, NH, NI, rp, m->dza, 1, NH, m->x, NI, 1, G + OFF_W1, nullptr, NI, nullptr, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, m->dza, rp, NH, G + OFF_B1);
    MLPCHK(hipGetLastError());
    return SHAKEN_OK;
}

shaken_status shaken_mlp_backward(shaken_mlp *m, const float *dy_dev, int32_t batch) {
    if (!m || !dy_dev) return set_error(SHAKEN_EINVAL, "need the network and dy");
    if (batch != m->rows || m->rows == 0) return set_error(SHAKEN_ESTATE, "backward needs the batch of the last forward");
    Dev guard(m->device);
    MLPCHK(hipMemsetAsync(m->dy, 0, (size_t)m->rows_pad * NO * 4, m->stream));
    MLPCHK(hipMemcpyAsync(m->dy, dy_dev, (size_t)batch * NO * 4, hipMemcpyDeviceToDevice, m->stream));
    return mlp_backward_from(m);
}

shaken_status shaken_mlp_loss_backward(shaken_mlp *m, const float *target_dev, const float *w_dev,
                                       int32_t batch, float *loss_host) {
    if (!m || !target_dev) return set_error(SHAKEN_EINVAL, "need the network and the targets");
    if (batch != m->rows || m->rows == 0) return set_error(SHAKEN_ESTATE, "loss needs the batch of the last forward");
    Dev guard(m->device);
    hipStream_t s = m->stream;
    hipLaunchKernelGGL(k_weight_sum, dim3(1), dim3(1024), 0, s, w_dev, batch, m->ws);
    MLPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_mse_grad, dim3(blocks((size_t)m->rows_pad * NO, 256)), dim3(256), 0, s, m->yf,
                       target_dev, w_dev, batch, m->rows_pad, m->ws, m->dy);
    MLPCHK(hipGetLastError());
    shaken_status st = mlp_backward_from(m);
    if (st != SHAKEN_OK) return st;
    if (loss_host) {
        float buf[2];
        MLPCHK(hipMemcpyAsync(buf, m->ws, 8, hipMemcpyDeviceToHost, s));
        MLPCHK(hipStreamSynchronize(s));
        *loss_host = buf[1];
    }
    return SHAKEN_OK;
}

shaken_status shaken_mlp_adam(shaken_mlp *m, float lr, float beta1, float beta2, float eps, int32_t t) {
    if (!m || t < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return set_error(SHAKEN_EINVAL, "bad Adam hyper-parameters");
    Dev guard(m->device);
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(blocks(NPARAM, 256)), dim3(256), 0, m->stream, m->w, m->g, m->m1, m->m2, m->wb,
                       (int)NPARAM, lr, beta1, beta2, eps, c1, c2);
    MLPCHK(hipGetLastError());
    return SHAKEN_OK;
}

}  // extern "C"

namespace shaken {
int mlp_device(const shaken_mlp *m) { return m->device; }
hipStream_t mlp_stream(const shaken_mlp *m) { return m->stream; }
}  // namespace shaken
