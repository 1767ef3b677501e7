// The learned PST proposal network: forward, Gaussian-NLL backward and Adam,
// with BF16 matrix-core (MFMA) GEMMs and FP32 accumulation.
//
// Parameters live in one caller-owned float32 buffer laid out
// [W1 (in x hid), b1 (hid), W2 (hid x hid), b2 (hid), W3 (hid x out), b3 (out)]
// (row-vector convention, y = x W + b); gradients and Adam moments use the
// same layout.  Operands are rounded to BF16 (round to nearest even) as the
// GEMM tiles are staged in LDS; products accumulate in FP32.
#include "common.h"

namespace rose {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ inline unsigned short to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_GELU_GRAD = 3 };

struct GemmArgs {
    int32_t M, N, K;
    const float* A;
    int64_t sam, sak;  // A(m, k) = A[m * sam + k * sak]
    const float* B;
    int64_t sbk, sbn;  // B(k, n) = B[k * sbk + n * sbn]
    float* C;
    int64_t ldc;       // C(m, n) = C[m * ldc + n]
    const float* bias; // EPI_BIAS*, length N
    float* H;          // EPI_BIAS_GELU: GELU(C), same layout as C
    const float* Z;    // EPI_GELU_GRAD: pre-activations, same layout as C
    int32_t mode;
};

constexpr int kGT = 64;  // block tile (M and N)
constexpr int kKT = 32;  // K tile
constexpr int kKP = kKT + 8;  // LDS row pitch (elements): 80-byte rows keep 16-byte reads aligned

// 256 threads = 2x2 wavefronts, each owning a 32x32 sub-tile computed with
// gfx950's double-K v_mfma_f32_32x32x16_bf16 (K = 16 per instruction).
// Operand layout: lane l holds A[l % 32][8 (l / 32) .. +7] and
// B[8 (l / 32) .. +7][l % 32]; the 16 accumulators of lane l are
// D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) unsigned short As[kGT][kKP];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[kGT][kKP];  // transposed: [n][k]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    f32x16_t acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    for (int k0 = 0; k0 < g.K; k0 += kKT) {
        for (int e = threadIdx.x; e < kGT * kKT; e += 256) {
            const int r = e / kKT, c = e % kKT;
            const int m = m0 + r, k = k0 + c;
            As[r][c] = to_bf16((m < g.M && k < g.K) ? g.A[m * g.sam + k * g.sak] : 0.0f);
        }
        for (int e = threadIdx.x; e < kGT * kKT; e += 256) {
            const int c = e / kGT, r = e % kGT;  // consecutive threads walk n
            const int n = n0 + r, k = k0 + c;
            Bs[r][c] = to_bf16((n < g.N && k < g.K) ? g.B[k * g.sbk + n * g.sbn] : 0.0f);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKT; kk += 16) {
            const int ml = wm * 32 + (lane & 31), nl = wn * 32 + (lane & 31), kb = kk + 8 * (lane >> 5);
            bf16x8_t a, b;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                a[q] = __builtin_bit_cast(__bf16, As[ml][kb + q]);
                b[q] = __builtin_bit_cast(__bf16, Bs[nl][kb + q]);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = m0 + wm * 32 + 8 * (i / 4) + 4 * (lane >> 5) + (i % 4);
        const int n = n0 + wn * 32 + (lane & 31);
        if (m >= g.M || n >= g.N) continue;
        const int64_t o = m * g.ldc + n;
        const float v = acc[i];
        if (g.mode == EPI_STORE) {
            g.C[o] = v;
        } else if (g.mode == EPI_BIAS_GELU) {
            const float z = v + g.bias[n];
            g.C[o] = z;
            g.H[o] = gelu_f(z);
        } else if (g.mode == EPI_BIAS) {
            g.C[o] = v + g.bias[n];
        } else {
            g.C[o] = v * gelu_grad_f(g.Z[o]);
        }
    }
}

// Gaussian NLL per sample and its gradient w.r.t. the 12 outputs (scaled by
// 1/B); one block reduces the per-sample losses in a fixed order.
__global__ __launch_bounds__(256) void k_nll(const float* out, const float* Y, int32_t B, float* dout, float* loss) {
    __shared__ double part[256];
    double s = 0.0;
    const float invB = 1.0f / (float)B;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        double lb = 0.0;
        for (int d = 0; d < 6; ++d) {
            const float mu = out[b * 12 + d], ls = out[b * 12 + 6 + d];
            const float r = Y[b * 6 + d] - mu;
            const float inv = expf(-2.0f * ls);
            lb += (double)(0.5f * r * r * inv + ls);
            dout[b * 12 + d] = -r * inv * invB;
            dout[b * 12 + 6 + d] = (1.0f - r * r * inv) * invB;
        }
        s += lb;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
        *loss = (float)(t / (double)B);
    }
}

// column sums (bias gradients): a workgroup per 64 columns; wave w of its
// 16 sums rows w, w + 16, ... of its lane's column (each row read as one
// coalesced 64-column segment), then one lane per column adds the 16
// partial sums in wave order (a fixed order: deterministic)
constexpr int kColsumWaves = 16;
__global__ __launch_bounds__(1024) void k_colsum(const float* X, int32_t rows, int32_t cols, float* out) {
    __shared__ float part[kColsumWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (c < cols)
        for (int r = w; r < rows; r += kColsumWaves) s += X[(int64_t)r * cols + c];
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && c < cols) {
        float t = 0.0f;
        for (int k = 0; k < kColsumWaves; ++k) t += part[k][lane];
        out[c] = t;
    }
}

__global__ __launch_bounds__(256) void k_adam(int64_t n, float* p, const float* gr, float* m, float* v, float lr,
                                             float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static rose_status gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                        int64_t sbn, float* C, int64_t ldc, int mode, const float* bias, float* H, const float* Z,
                        hipStream_t s) {
    GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, H, Z, mode};
    dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

}  // namespace rose

struct rose_mlp {
    int32_t in, hid, out, max_batch;
    float *Z1, *H1, *Z2, *H2, *Y, *dY, *dZ2, *dZ1, *dH;
};

using namespace rose;

namespace {
struct Offs {
    int64_t W1, b1, W2, b2, W3, b3, total;
};
Offs offsets(int in, int hid, int out) {
    Offs o;
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)in * hid;
    o.W2 = o.b1 + hid;
    o.b2 = o.W2 + (int64_t)hid * hid;
    o.W3 = o.b2 + hid;
    o.b3 = o.W3 + (int64_t)hid * out;
    o.total = o.b3 + out;
    return o;
}
}  // namespace

extern "C" {

int64_t rose_mlp_param_count(int32_t in_dim, int32_t hidden, int32_t out_dim) {
    if (in_dim < 1 || hidden < 1 || out_dim != 12) return 0;
    return offsets(in_dim, hidden, out_dim).total;
}

rose_status rose_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, int32_t max_batch, rose_mlp** out) {
    clear_error();
    ROSE_REQUIRE(out != nullptr, ROSE_E_ARG, "rose_mlp_create: NULL output");
    *out = nullptr;
    ROSE_REQUIRE(in_dim >= 1 && in_dim <= 65536 && hidden >= 1 && hidden <= 4096 && out_dim == 12 &&
                     max_batch >= 1 && max_batch <= 65536,
                 ROSE_E_SHAPE, "rose_mlp_create: sizes out of range (out_dim must be 12)");
    rose_mlp* m = (rose_mlp*)calloc(1, sizeof(rose_mlp));
    ROSE_REQUIRE(m != nullptr, ROSE_E_DEVICE, "rose_mlp_create: out of host memory");
    m->in = in_dim;
    m->hid = hidden;
    m->out = out_dim;
    m->max_batch = max_batch;
    const size_t bh = sizeof(float) * (size_t)max_batch * hidden;
    const size_t bo = sizeof(float) * (size_t)max_batch * out_dim;
    float** bufs_h[] = {&m->Z1, &m->H1, &m->Z2, &m->H2, &m->dZ2, &m->dZ1, &m->dH};
    bool ok = true;
    for (float** b : bufs_h) ok = ok && hipMalloc((void**)b, bh) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->Y, bo) == hipSuccess && hipMalloc((void**)&m->dY, bo) == hipSuccess;
    if (!ok) {
        rose_mlp_destroy(m);
        set_error("rose_mlp_create: hipMalloc failed");
        return ROSE_E_DEVICE;
    }
    *out = m;
    return ROSE_OK;
}

rose_status rose_mlp_destroy(rose_mlp* m) {
    clear_error();
    if (!m) return ROSE_OK;
    (void)hipDeviceSynchronize();
    float* bufs[] = {m->Z1, m->H1, m->Z2, m->H2, m->Y, m->dY, m->dZ2, m->dZ1, m->dH};
    for (float* b : bufs)
        if (b) (void)hipFree(b);
    free(m);
    return ROSE_OK;
}

static rose_status mlp_forward_impl(rose_mlp* m, const float* P, const float* X, int32_t B, float* out,
                                    hipStream_t s) {
    const Offs o = offsets(m->in, m->hid, m->out);
    rose_status st;
    if ((st = gemm(B, m->hid, m->in, X, m->in, 1, P + o.W1, m->hid, 1, m->Z1, m->hid, EPI_BIAS_GELU, P + o.b1,
                   m->H1, nullptr, s)) != ROSE_OK)
        return st;
    if ((st = gemm(B, m->hid, m->hid, m->H1, m->hid, 1, P + o.W2, m->hid, 1, m->Z2, m->hid, EPI_BIAS_GELU, P + o.b2,
                   m->H2, nullptr, s)) != ROSE_OK)
        return st;
    return gemm(B, m->out, m->hid, m->H2, m->hid, 1, P + o.W3, m->out, 1, out, m->out, EPI_BIAS, P + o.b3, nullptr,
                nullptr, s);
}

rose_status rose_mlp_forward(rose_mlp* m, const float* params_dev, const float* X_dev, int32_t B, float* out_dev,
                             hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(m && params_dev && X_dev && out_dev, ROSE_E_ARG, "rose_mlp_forward: NULL argument");
    ROSE_REQUIRE(B >= 1 && B <= m->max_batch, ROSE_E_SHAPE, "rose_mlp_forward: batch %d out of [1, %d]", B,
                 m->max_batch);
    return mlp_forward_impl(m, params_dev, X_dev, B, out_dev, s);
}

rose_status rose_mlp_loss_grad(rose_mlp* m, const float* params_dev, const float* X_dev, const float* Y_dev,
                               int32_t B, float* grads_dev, float* loss_dev, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(m && params_dev && X_dev && Y_dev && grads_dev && loss_dev, ROSE_E_ARG,
                 "rose_mlp_loss_grad: NULL argument");
    ROSE_REQUIRE(B >= 1 && B <= m->max_batch, ROSE_E_SHAPE, "rose_mlp_loss_grad: batch %d out of [1, %d]", B,
                 m->max_batch);
    const Offs o = offsets(m->in, m->hid, m->out);
    const float* P = params_dev;
    float* G = grads_dev;
    rose_status st;
    if ((st = mlp_forward_impl(m, P, X_dev, B, m->Y, s)) != ROSE_OK) return st;
    hipLaunchKernelGGL(k_nll, dim3(1), dim3(256), 0, s, m->Y, Y_dev, B, m->dY, loss_dev);
    ROSE_CHECK_HIP(hipGetLastError());
    const int hid = m->hid, in = m->in, out = m->out;
    // dW3 = H2^T dY ; db3 = colsum(dY)
    if ((st = gemm(hid, out, B, m->H2, 1, hid, m->dY, out, 1, G + o.W3, out, EPI_STORE, nullptr, nullptr, nullptr,
                   s)) != ROSE_OK)
        return st;
    hipLaunchKernelGGL(k_colsum, dim3((out + 63) / 64), dim3(64 * kColsumWaves), 0, s, m->dY, B, out, G + o.b3);
    // dZ2 = (dY W3^T) * gelu'(Z2)
    if ((st = gemm(B, hid, out, m->dY, out, 1, P + o.W3, 1, out, m->dZ2, hid, EPI_GELU_GRAD, nullptr, nullptr, m->Z2,
                   s)) != ROSE_OK)
        return st;
    // dW2 = H1^T dZ2 ; db2
    if ((st = gemm(hid, hid, B, m->H1, 1, hid, m->dZ2, hid, 1, G + o.W2, hid, EPI_STORE, nullptr, nullptr, nullptr,
                   s)) != ROSE_OK)
        return st;
    hipLaunchKernelGGL(k_colsum, dim3((hid + 63) / 64), dim3(64 * kColsumWaves), 0, s, m->dZ2, B, hid, G + o.b2);
    // dZ1 = (dZ2 W2^T) * gelu'(Z1)
    if ((st = gemm(B, hid, hid, m->dZ2, hid, 1, P + o.W2, 1, hid, m->dZ1, hid, EPI_GELU_GRAD, nullptr, nullptr, m->Z1,
                   s)) != ROSE_OK)
        return st;
    // dW1 = X^T dZ1 ; db1
    if ((st = gemm(in, hid, B, X_dev, 1, in, m->dZ1, hid, 1, G + o.W1, hid, EPI_STORE, nullptr, nullptr, nullptr,
                   s)) != ROSE_OK)
        return st;
    hipLaunchKernelGGL(k_colsum, dim3((hid + 63) / 64), dim3(64 * kColsumWaves), 0, s, m->dZ1, B, hid, G + o.b1);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status rose_mlp_adam(int64_t n, float* params_dev, const float* grads_dev, float* m_dev, float* v_dev,
                          int32_t step, float lr, float beta1, float beta2, float eps, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(params_dev && grads_dev && m_dev && v_dev, ROSE_E_ARG, "rose_mlp_adam: NULL argument");
    ROSE_REQUIRE(n >= 1 && step >= 1, ROSE_E_ARG, "rose_mlp_adam: n >= 1 and step >= 1 required");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, params_dev, grads_dev, m_dev,
                       v_dev, lr, beta1, beta2, eps, c1, c2);
    ROSE_CHECK_HIP(hipGetLastError());
    return ROSE_OK;
}

rose_status rose_gemm_bf16(int32_t M, int32_t N, int32_t K, const float* A_dev, int64_t sam, int64_t sak,
                           const float* B_dev, int64_t sbk, int64_t sbn, float* C_dev, int64_t ldc, hipStream_t s) {
    clear_error();
    ROSE_REQUIRE(A_dev && B_dev && C_dev, ROSE_E_ARG, "rose_gemm_bf16: NULL argument");
    ROSE_REQUIRE(M >= 1 && N >= 1 && K >= 1 && M <= 65536 && N <= 65536 && K <= 65536, ROSE_E_SHAPE,
                 "rose_gemm_bf16: sizes out of range");
    return gemm(M, N, K, A_dev, sam, sak, B_dev, sbk, sbn, C_dev, ldc, EPI_STORE, nullptr, nullptr, nullptr, s);
}

}  // extern "C"
