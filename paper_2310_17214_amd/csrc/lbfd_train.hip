// lbfd_train.hip -- training of the chemistry surrogate on one GPU.
//
// Mini-batch Adam on the mean-square error of the standardised outputs of the
// perceptron n_in -> 256 -> 256 -> n_out (ReLU).  FP32 master weights and
// moments; forward and backward products on the matrix cores with bf16
// operands and FP32 accumulation, all written as C = A B^T with both operands
// K-contiguous ("NT"), so every fragment is one 16-byte load:
//   forward    Z1 = W1 X^T, Z2 = W2 H1^T, Yh = W3 H2^T          (samples = N)
//   backward   D2^T = W3^T D3^T (.) [H2 > 0],  D1^T = W2^T D2^T (.) [H1 > 0]
//   gradients  dW2 = D2f H1f^T, dW1 = D1f Xf^T, dW3 = D3f H2f^T  (K = samples,
//              split into slices of 256 and summed in a fixed order)
// Activations are stored sample-major ([n][feature], the next product's B
// operand) and feature-major ([feature][n], the gradient products'
// operands).  Every reduction has a fixed order, so a step is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbfd.h"
#include "lbfd_mlp.h"

namespace lbfd {
namespace {

constexpr int TB = 256;   // threads per workgroup
constexpr int KS = 256;   // K slice of the split gradient products
constexpr int H = MLP_H;

struct TrainNorm {
    float mu_x[MLP_KIN], sd_x[MLP_KIN], inv_sd_x[MLP_KIN], lo[MLP_KIN], hi[MLP_KIN];
    float mu_y[MLP_OUT], sd_y[MLP_OUT], inv_sd_y[MLP_OUT];
};

typedef unsigned short u16;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u16 bf16_bits(float v) {
    const __bf16 b = (__bf16)v;
    return __builtin_bit_cast(u16, b);
}
__device__ __forceinline__ float bf16_float(u16 b) {
    return __uint_as_float((unsigned)b << 16);
}

// ------------------------------------------------------------ statistics
// One workgroup per column (inputs first, then targets): FP64 mean, then
// population standard deviation (floored at 1e-12 max(|mu|, 1), and at 1e-4
// for the mass-fraction inputs), min, max.
__global__ __launch_bounds__(TB) void norm_fit_kernel(const float* __restrict__ x,
                                                      const float* __restrict__ y, int n, int ni,
                                                      int no, TrainNorm* __restrict__ out) {
    __shared__ double s1[TB], s2[TB], s3[TB];
    const int c = blockIdx.x, t = threadIdx.x;
    const bool isx = c < ni;
    const float* col = isx ? x + c : y + (c - ni);
    const int stride = isx ? ni : no;
    double a = 0.0;
    for (int i = t; i < n; i += TB) a += (double)col[(size_t)i * stride];
    s1[t] = a;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if (t < w) s1[t] += s1[t + w];
        __syncthreads();
    }
    const double mu = s1[0] / (double)n;
    double v = 0.0, lo = 1e300, hi = -1e300;
    for (int i = t; i < n; i += TB) {
        const double d = (double)col[(size_t)i * stride];
        v += (d - mu) * (d - mu);
        lo = fmin(lo, d);
        hi = fmax(hi, d);
    }
    s1[t] = v;
    s2[t] = lo;
    s3[t] = hi;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if (t < w) {
            s1[t] += s1[t + w];
            s2[t] = fmin(s2[t], s2[t + w]);
            s3[t] = fmax(s3[t], s3[t + w]);
        }
        __syncthreads();
    }
    if (t == 0) {
        double sd = sqrt(s1[0] / (double)n);
        sd = fmax(sd, 1e-12 * fmax(fabs(mu), 1.0));
        // mass-fraction inputs: species that stay below ~1e-4 are seen as
        // near-constant inputs rather than amplified by a tiny spread
        if (isx && c >= 2) sd = fmax(sd, 1e-4);
        if (isx) {
            out->mu_x[c] = (float)mu;
            out->sd_x[c] = (float)sd;
            out->inv_sd_x[c] = (float)(1.0 / sd);
            out->lo[c] = (float)s2[0];
            out->hi[c] = (float)s3[0];
        } else {
            const int o = c - ni;
            out->mu_y[o] = (float)mu;
            out->sd_y[o] = (float)sd;
            out->inv_sd_y[o] = (float)(1.0 / sd);
        }
    }
}

// ----------------------------------------------------------------- batch
// Gather the batch rows idx[0..B) and standardise: Xs [B][16], Xf [32][B]
// (bf16, features past n_in zero), Tt [B][16] (FP32 targets, past n_out
// zero).  Indices outside [0, n) give zero rows.
__global__ __launch_bounds__(TB) void prep_kernel(const float* __restrict__ x,
                                                  const float* __restrict__ y, int n,
                                                  const int* __restrict__ idx, int B, int ni,
                                                  int no, const TrainNorm* __restrict__ nm,
                                                  u16* __restrict__ Xs, u16* __restrict__ Xf,
                                                  float* __restrict__ Tt) {
    const int s = blockIdx.x * TB + threadIdx.x;
    if (s >= B) return;
    const int i = idx[s];
    const bool ok = i >= 0 && i < n;
    for (int f = 0; f < 32; ++f) {
        float v = 0.f;
        if (ok && f < ni) v = (x[(size_t)i * ni + f] - nm->mu_x[f]) * nm->inv_sd_x[f];
        const u16 b = f < ni ? bf16_bits(v) : (u16)0;
        if (f < MLP_KIN) Xs[(size_t)s * MLP_KIN + f] = b;
        Xf[(size_t)f * B + s] = b;
    }
    for (int o = 0; o < MLP_OUT; ++o) {
        float v = 0.f;
        if (ok && o < no) v = (y[(size_t)i * no + o] - nm->mu_y[o]) * nm->inv_sd_y[o];
        Tt[(size_t)s * MLP_OUT + o] = v;
    }
}

// ------------------------------------------------------------ NT product
enum { EPI_HID = 0, EPI_OUT = 1, EPI_MASK = 2, EPI_PART = 3 };

struct Gemm {
    const u16* A;  // [M][lda], K-contiguous
    const u16* B;  // [N][ldb], K-contiguous
    int lda, ldb, M, N, K, kslice;
    // epilogue
    const float* bias;   // [M] (HID, OUT)
    int mvalid;          // rows < mvalid are real (OUT)
    const u16* mask_s;   // [N][M] sample-major ReLU reference (MASK)
    u16* out_s;          // [N][lds] sample-major bf16 (HID, OUT, MASK; may be null)
    int lds;
    u16* out_f;          // [M][N] feature-major bf16 (HID, OUT, MASK)
    const float* target; // [N][16] standardised targets (OUT)
    float gscale;        // 2 / (B n_out) (OUT)
    double* loss_part;   // [N / 32] (OUT)
    float* part;         // [S][M][N] (PART)
};

// One wave per 32 x 32 tile of C (and K slice); accumulator r of lane l is
// C[8 (r/4) + 4 (l/32) + r%4][l%32] of the tile.
template <int EPI>
__global__ __launch_bounds__(TB) void gemm_nt_kernel(Gemm g) {
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int w = blockIdx.x * (TB / 64) + (threadIdx.x >> 6);
    const int tm = g.M / 32, tn = g.N / 32, S = g.K / g.kslice;
    if (w >= tm * tn * S) return;  // whole wave
    const int im = w % tm, rest = w / tm, in = rest % tn, ks = rest / tn;
    const int m0 = im * 32, n0 = in * 32;
    const u16* ap = g.A + (size_t)(m0 + lane % 32) * g.lda + 8 * h;
    const u16* bp = g.B + (size_t)(n0 + lane % 32) * g.ldb + 8 * h;
    f32x16 acc = {};
    const int k0 = ks * g.kslice, k1 = k0 + g.kslice;
#pragma unroll 4
    for (int k = k0; k < k1; k += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap + k);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(bp + k);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    const int n = n0 + lane % 32;
    if constexpr (EPI == EPI_PART) {
        float* p = g.part + (size_t)ks * g.M * g.N;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = m0 + 8 * (r / 4) + 4 * h + r % 4;
            p[(size_t)i * g.N + n] = acc[r];
        }
        return;
    }
    double lsum = 0.0;
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
        const int i0 = m0 + 8 * gq + 4 * h;  // rows i0 .. i0 + 3
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = i0 + j;
            float c = acc[4 * gq + j];
            if constexpr (EPI == EPI_HID) {
                c = fmaxf(c + g.bias[i], 0.f);
            } else if constexpr (EPI == EPI_OUT) {
                if (i < g.mvalid) {
                    const float yh = c + g.bias[i];
                    const float d = yh - g.target[(size_t)n * MLP_OUT + i];
                    lsum += (double)d * (double)d;
                    c = g.gscale * d;
                } else {
                    c = 0.f;
                }
            } else if constexpr (EPI == EPI_MASK) {
                const u16 ref = g.mask_s[(size_t)n * g.M + i];
                c = ((short)ref > 0) ? c : 0.f;
            }
            v[j] = c;
        }
        u16 b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = bf16_bits(v[j]);
        if (g.out_s && (EPI != EPI_OUT || i0 < MLP_OUT)) {
            u16* o = g.out_s + (size_t)n * g.lds + i0;
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = b[j];
        }
        if (g.out_f) {
#pragma unroll
            for (int j = 0; j < 4; ++j) g.out_f[(size_t)(i0 + j) * g.N + n] = b[j];
        }
    }
    if constexpr (EPI == EPI_OUT) {
        // per-tile loss: fixed-order reduction over the wave's lanes via LDS-free shuffles
        for (int o = 32; o >= 1; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        if (lane == 0) g.loss_part[w] = lsum;
    }
}

// ------------------------------------------------------------ reductions
// out[off + i * cols + j] = sum_s part[s][i][j] (i < rows, j < cols; the part
// planes are [Mp][Np]).
__global__ __launch_bounds__(TB) void part_sum_kernel(const float* __restrict__ part, int S,
                                                      int Mp, int Np, int rows, int cols,
                                                      float* __restrict__ out) {
    const int t = blockIdx.x * TB + threadIdx.x;
    if (t >= rows * cols) return;
    const int i = t / cols, j = t % cols;
    double a = 0.0;
    for (int s = 0; s < S; ++s) a += (double)part[((size_t)s * Mp + i) * Np + j];
    out[t] = (float)a;
}

// out[i] = sum_n D[i][n] (bf16 rows of length N), one workgroup per row.
__global__ __launch_bounds__(TB) void row_sum_kernel(const u16* __restrict__ D, int N,
                                                     float* __restrict__ out) {
    __shared__ double s[TB];
    const int i = blockIdx.x, t = threadIdx.x;
    double a = 0.0;
    for (int n = t; n < N; n += TB) a += (double)bf16_float(D[(size_t)i * N + n]);
    s[t] = a;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    if (t == 0) out[i] = (float)s[0];
}

__global__ __launch_bounds__(TB) void loss_sum_kernel(const double* __restrict__ part, int n,
                                                      double scale, double* __restrict__ out) {
    __shared__ double s[TB];
    const int t = threadIdx.x;
    double a = 0.0;
    for (int i = t; i < n; i += TB) a += part[i];
    s[t] = a;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    if (t == 0) *out = s[0] * scale;
}

// ------------------------------------------------------------ update
// Adam (Kingma and Ba): c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
__global__ __launch_bounds__(TB) void adam_kernel(float* __restrict__ w, float* __restrict__ m,
                                                  float* __restrict__ v,
                                                  const float* __restrict__ g, int n, float lr,
                                                  float b1, float b2, float eps, float c1,
                                                  float c2) {
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// bf16 operand copies of the master weights: W1b [256][16], W2b [256][256],
// W3b [32][256], W3Tb [256][16], W2Tb [256][256] (zero padding).
__global__ __launch_bounds__(TB) void pack_kernel(const float* __restrict__ P, int ni, int no,
                                                  u16* __restrict__ W1b, u16* __restrict__ W2b,
                                                  u16* __restrict__ W3b, u16* __restrict__ W3Tb,
                                                  u16* __restrict__ W2Tb) {
    const int t = blockIdx.x * TB + threadIdx.x;
    const float* W1 = P;
    const float* W2 = W1 + H * ni + H;
    const float* W3 = W2 + H * H + H;
    if (t < H * H) {
        const int i = t / H, k = t % H;
        W2b[t] = bf16_bits(W2[t]);
        W2Tb[(size_t)k * H + i] = bf16_bits(W2[t]);
    }
    if (t < H * MLP_KIN) {
        const int i = t / MLP_KIN, f = t % MLP_KIN;
        W1b[t] = f < ni ? bf16_bits(W1[i * ni + f]) : (u16)0;
        W3Tb[t] = f < no ? bf16_bits(W3[f * H + i]) : (u16)0;  // [i][o]
    }
    if (t < 32 * H) {
        const int o = t / H, i = t % H;
        W3b[t] = o < no ? bf16_bits(W3[o * H + i]) : (u16)0;
    }
}

}  // namespace
}  // namespace lbfd

using namespace lbfd;

struct TrainLayout {
    size_t P, M, V, G, norm, W1b, W2b, W3b, W3Tb, W2Tb, Xs, Xf, Tt, H1s, H1f, H2s, H2f, D3s, D3f,
        D2s, D2f, D1f, p1, p2, p3, lossp, loss, total;
};

struct lbfd_trainer {
    lbfd_train_cfg cfg;
    TrainLayout L;
    int ni, no, np;
    char* ws;
    hipStream_t stream;
    int device;
    int64_t t = 0;
    bool have_norm = false, have_w = false;
    std::string err;
};

namespace {

int n_params(int ni, int no) { return H * ni + H + H * H + H + no * H + no; }

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

TrainLayout train_layout(const lbfd_train_cfg& c) {
    TrainLayout L;
    const size_t B = (size_t)c.batch, S = B / KS;
    const int ni = 2 + c.n_species, no = c.n_species, np = n_params(ni, no);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = al(off + bytes);
        return o;
    };
    L.P = take(np * 4);
    L.M = take(np * 4);
    L.V = take(np * 4);
    L.G = take(np * 4);
    L.norm = take(sizeof(TrainNorm));
    L.W1b = take(H * MLP_KIN * 2);
    L.W2b = take(H * H * 2);
    L.W3b = take(32 * H * 2);
    L.W3Tb = take(H * MLP_KIN * 2);
    L.W2Tb = take(H * H * 2);
    L.Xs = take(B * MLP_KIN * 2);
    L.Xf = take(32 * B * 2);
    L.Tt = take(B * MLP_OUT * 4);
    L.H1s = take(B * H * 2);
    L.H1f = take(B * H * 2);
    L.H2s = take(B * H * 2);
    L.H2f = take(B * H * 2);
    L.D3s = take(B * MLP_OUT * 2);
    L.D3f = take(32 * B * 2);
    L.D2s = take(B * H * 2);
    L.D2f = take(B * H * 2);
    L.D1f = take(B * H * 2);
    L.p1 = take(S * H * 32 * 4);
    L.p2 = take(S * H * H * 4);
    L.p3 = take(S * 32 * H * 4);
    L.lossp = take((B / 32) * 8);
    L.loss = take(8);
    L.total = off;
    return L;
}

lbfd_status check_cfg(const lbfd_train_cfg* c) {
    if (!c) return LBFD_E_INVAL;
    if (c->n_species < 1 || c->n_species + 2 > MLP_KIN) return LBFD_E_UNSUPPORTED;
    if (c->batch < KS || c->batch % KS != 0 || c->batch > (1 << 22)) return LBFD_E_INVAL;
    if (!(c->beta1 >= 0.f && c->beta1 < 1.f && c->beta2 >= 0.f && c->beta2 < 1.f &&
          c->eps > 0.f))
        return LBFD_E_INVAL;
    return LBFD_OK;
}

lbfd_status tfail(lbfd_trainer* t, lbfd_status st, const std::string& m) {
    if (t) t->err = m;
    return st;
}
lbfd_status thip(lbfd_trainer* t, hipError_t e, const char* what) {
    if (e == hipSuccess) return LBFD_OK;
    return tfail(t, LBFD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
template <typename T>
T* tp(lbfd_trainer* t, size_t off) {
    return reinterpret_cast<T*>(t->ws + off);
}

template <int EPI>
hipError_t gemm(lbfd_trainer* t, const Gemm& g) {
    const int waves = (g.M / 32) * (g.N / 32) * (g.K / g.kslice);
    hipLaunchKernelGGL((gemm_nt_kernel<EPI>), dim3((waves + 3) / 4), dim3(TB), 0, t->stream, g);
    return hipGetLastError();
}

// Forward and backward of one batch: gradient into G, mean loss into `loss`.
lbfd_status forward_backward(lbfd_trainer* t, const float* x, const float* y, int n,
                             const int* idx) {
    const int B = t->cfg.batch, ni = t->ni, no = t->no, S = B / KS;
    const float* P = tp<float>(t, t->L.P);
    const float* b1 = P + H * ni;
    const float* b2 = b1 + H + H * H;
    const float* b3 = b2 + H + no * H;
    float* G = tp<float>(t, t->L.G);
    hipError_t e;
    hipLaunchKernelGGL(prep_kernel, dim3((B + TB - 1) / TB), dim3(TB), 0, t->stream, x, y, n, idx,
                       B, ni, no, tp<TrainNorm>(t, t->L.norm), tp<u16>(t, t->L.Xs),
                       tp<u16>(t, t->L.Xf), tp<float>(t, t->L.Tt));
    if ((e = hipGetLastError()) != hipSuccess) return thip(t, e, "prep");
    Gemm g;
    std::memset(&g, 0, sizeof(g));
    // Z1 = W1 X^T -> H1
    g.A = tp<u16>(t, t->L.W1b); g.lda = MLP_KIN;
    g.B = tp<u16>(t, t->L.Xs); g.ldb = MLP_KIN;
    g.M = H; g.N = B; g.K = MLP_KIN; g.kslice = MLP_KIN;
    g.bias = b1; g.out_s = tp<u16>(t, t->L.H1s); g.lds = H; g.out_f = tp<u16>(t, t->L.H1f);
    if ((e = gemm<EPI_HID>(t, g)) != hipSuccess) return thip(t, e, "forward 1");
    // Z2 = W2 H1^T -> H2
    g.A = tp<u16>(t, t->L.W2b); g.lda = H;
    g.B = tp<u16>(t, t->L.H1s); g.ldb = H;
    g.K = H; g.kslice = H;
    g.bias = b2; g.out_s = tp<u16>(t, t->L.H2s); g.out_f = tp<u16>(t, t->L.H2f);
    if ((e = gemm<EPI_HID>(t, g)) != hipSuccess) return thip(t, e, "forward 2");
    // Yh = W3 H2^T -> D3 = 2 (Yh - T)/(B n_out), per-tile loss
    g.A = tp<u16>(t, t->L.W3b);
    g.B = tp<u16>(t, t->L.H2s);
    g.M = 32;
    g.bias = b3; g.mvalid = no;
    g.target = tp<float>(t, t->L.Tt);
    g.gscale = 2.f / ((float)B * (float)no);
    g.out_s = tp<u16>(t, t->L.D3s); g.lds = MLP_OUT; g.out_f = tp<u16>(t, t->L.D3f);
    g.loss_part = tp<double>(t, t->L.lossp);
    if ((e = gemm<EPI_OUT>(t, g)) != hipSuccess) return thip(t, e, "forward 3");
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(TB), 0, t->stream,
                       tp<double>(t, t->L.lossp), B / 32, 1.0 / ((double)B * no),
                       tp<double>(t, t->L.loss));
    if ((e = hipGetLastError()) != hipSuccess) return thip(t, e, "loss");
    // D2^T = W3^T D3^T masked by H2
    std::memset(&g, 0, sizeof(g));
    g.A = tp<u16>(t, t->L.W3Tb); g.lda = MLP_KIN;
    g.B = tp<u16>(t, t->L.D3s); g.ldb = MLP_OUT;
    g.M = H; g.N = B; g.K = MLP_OUT; g.kslice = MLP_OUT;
    g.mask_s = tp<u16>(t, t->L.H2s);
    g.out_s = tp<u16>(t, t->L.D2s); g.lds = H; g.out_f = tp<u16>(t, t->L.D2f);
    if ((e = gemm<EPI_MASK>(t, g)) != hipSuccess) return thip(t, e, "backward 2");
    // D1^T = W2^T D2^T masked by H1
    g.A = tp<u16>(t, t->L.W2Tb); g.lda = H;
    g.B = tp<u16>(t, t->L.D2s); g.ldb = H;
    g.K = H; g.kslice = H;
    g.mask_s = tp<u16>(t, t->L.H1s);
    g.out_s = nullptr; g.out_f = tp<u16>(t, t->L.D1f);
    if ((e = gemm<EPI_MASK>(t, g)) != hipSuccess) return thip(t, e, "backward 1");
    // weight gradients (split K over the batch)
    std::memset(&g, 0, sizeof(g));
    g.kslice = KS; g.K = B; g.lda = B; g.ldb = B;
    g.A = tp<u16>(t, t->L.D2f); g.B = tp<u16>(t, t->L.H1f); g.M = H; g.N = H;
    g.part = tp<float>(t, t->L.p2);
    if ((e = gemm<EPI_PART>(t, g)) != hipSuccess) return thip(t, e, "grad W2");
    g.A = tp<u16>(t, t->L.D1f); g.B = tp<u16>(t, t->L.Xf); g.M = H; g.N = 32;
    g.part = tp<float>(t, t->L.p1);
    if ((e = gemm<EPI_PART>(t, g)) != hipSuccess) return thip(t, e, "grad W1");
    g.A = tp<u16>(t, t->L.D3f); g.B = tp<u16>(t, t->L.H2f); g.M = 32; g.N = H;
    g.part = tp<float>(t, t->L.p3);
    if ((e = gemm<EPI_PART>(t, g)) != hipSuccess) return thip(t, e, "grad W3");
    float* gW1 = G;
    float* gb1 = gW1 + H * ni;
    float* gW2 = gb1 + H;
    float* gb2 = gW2 + H * H;
    float* gW3 = gb2 + H;
    float* gb3 = gW3 + no * H;
    auto psum = [&](size_t part, int Mp, int Np, int rows, int cols, float* out) {
        hipLaunchKernelGGL(part_sum_kernel, dim3((rows * cols + TB - 1) / TB), dim3(TB), 0,
                           t->stream, tp<float>(t, part), S, Mp, Np, rows, cols, out);
        return hipGetLastError();
    };
    if ((e = psum(t->L.p1, H, 32, H, ni, gW1)) != hipSuccess) return thip(t, e, "sum W1");
    if ((e = psum(t->L.p2, H, H, H, H, gW2)) != hipSuccess) return thip(t, e, "sum W2");
    if ((e = psum(t->L.p3, 32, H, no, H, gW3)) != hipSuccess) return thip(t, e, "sum W3");
    hipLaunchKernelGGL(row_sum_kernel, dim3(H), dim3(TB), 0, t->stream, tp<u16>(t, t->L.D1f), B,
                       gb1);
    hipLaunchKernelGGL(row_sum_kernel, dim3(H), dim3(TB), 0, t->stream, tp<u16>(t, t->L.D2f), B,
                       gb2);
    hipLaunchKernelGGL(row_sum_kernel, dim3(no), dim3(TB), 0, t->stream, tp<u16>(t, t->L.D3f), B,
                       gb3);
    if ((e = hipGetLastError()) != hipSuccess) return thip(t, e, "bias gradients");
    return LBFD_OK;
}

lbfd_status pack(lbfd_trainer* t) {
    hipLaunchKernelGGL(pack_kernel, dim3((H * H + TB - 1) / TB), dim3(TB), 0, t->stream,
                       tp<float>(t, t->L.P), t->ni, t->no, tp<u16>(t, t->L.W1b),
                       tp<u16>(t, t->L.W2b), tp<u16>(t, t->L.W3b), tp<u16>(t, t->L.W3Tb),
                       tp<u16>(t, t->L.W2Tb));
    return thip(t, hipGetLastError(), "pack");
}

// Statistics in the host layouts of lbfd_set_surrogate (either may be NULL).
void norm_to_host(const TrainNorm& nm, int ni, int no, float* norm, float* env) {
    if (norm) {
        for (int i = 0; i < ni; ++i) {
            norm[i] = nm.mu_x[i];
            norm[ni + i] = nm.sd_x[i];
        }
        for (int o = 0; o < no; ++o) {
            norm[2 * ni + o] = nm.mu_y[o];
            norm[2 * ni + no + o] = nm.sd_y[o];
        }
    }
    if (env) {
        for (int i = 0; i < ni; ++i) {
            env[i] = nm.lo[i];
            env[ni + i] = nm.hi[i];
        }
    }
}

// ------------------------------------------ statistics without allocation
// The statistics kernel of lbfd_trainer_fit_norm writes into a device-side
// staging block that, for lbfd_fit_norm_noalloc, is this file-scope array: one
// copy per GPU, alive until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is a stand-in, not a
// device address): it passes the address hipGetSymbolAddress returns for the
// current device, looked up once per device and kept in scratch_addr.
constexpr size_t NORM_SCRATCH_BYTES = 4096;  // one TrainNorm (16 inputs, 16 outputs)
static_assert(sizeof(TrainNorm) <= NORM_SCRATCH_BYTES, "statistics scratch");
static __device__ __align__(256) unsigned char scratch[NORM_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void* scratch_addr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device); nullptr and the HIP error otherwise.
void* scratch_for_device(int device, hipError_t* err) {
    *err = hipSuccess;
    if (device < 0 || device >= MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        scratch_addr[device] = p;
    }
    return scratch_addr[device];
}

lbfd_status batch_args(lbfd_trainer* t, const float* x, const float* y, int32_t n,
                       const int32_t* idx) {
    if (!x || !y || !idx || n < 1) return tfail(t, LBFD_E_INVAL, "data and batch indices");
    if (!t->have_norm || !t->have_w) return tfail(t, LBFD_E_STATE, "fit_norm and weights first");
    return thip(t, hipSetDevice(t->device), "hipSetDevice");
}

}  // namespace

extern "C" {

lbfd_status lbfd_trainer_workspace_bytes(const lbfd_train_cfg* cfg, size_t* bytes) {
    lbfd_status st = check_cfg(cfg);
    if (st) return st;
    if (!bytes) return LBFD_E_INVAL;
    *bytes = train_layout(*cfg).total;
    return LBFD_OK;
}

lbfd_status lbfd_trainer_create(const lbfd_train_cfg* cfg, void* ws, size_t bytes, void* stream,
                                lbfd_trainer** out) {
    if (!out) return LBFD_E_INVAL;
    *out = nullptr;
    lbfd_status st = check_cfg(cfg);
    if (st) return st;
    const TrainLayout L = train_layout(*cfg);
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0) return LBFD_E_INVAL;
    if (bytes < L.total) return LBFD_E_NOMEM;
    lbfd_trainer* t = new (std::nothrow) lbfd_trainer();
    if (!t) return LBFD_E_NOMEM;
    t->cfg = *cfg;
    t->L = L;
    t->ni = 2 + cfg->n_species;
    t->no = cfg->n_species;
    t->np = n_params(t->ni, t->no);
    t->ws = reinterpret_cast<char*>(ws);
    t->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&t->device) != hipSuccess) {
        delete t;
        return LBFD_E_DEVICE;
    }
    *out = t;
    return LBFD_OK;
}

lbfd_status lbfd_trainer_fit_norm(lbfd_trainer* t, const float* x, const float* y, int32_t n) {
    if (!t) return LBFD_E_INVAL;
    if (!x || !y || n < 2) return tfail(t, LBFD_E_INVAL, "need at least two samples");
    lbfd_status st = thip(t, hipSetDevice(t->device), "hipSetDevice");
    if (st) return st;
    hipLaunchKernelGGL(norm_fit_kernel, dim3(t->ni + t->no), dim3(TB), 0, t->stream, x, y, n,
                       t->ni, t->no, tp<TrainNorm>(t, t->L.norm));
    if ((st = thip(t, hipGetLastError(), "fit_norm"))) return st;
    t->have_norm = true;
    return LBFD_OK;
}

lbfd_status lbfd_trainer_set_weights(lbfd_trainer* t, const float* w) {
    if (!t || !w) return LBFD_E_INVAL;
    for (int i = 0; i < t->np; ++i)
        if (!std::isfinite(w[i])) return tfail(t, LBFD_E_INVAL, "non-finite weight");
    lbfd_status st = thip(t, hipSetDevice(t->device), "hipSetDevice");
    if (st) return st;
    const size_t nb = (size_t)t->np * 4;
    if ((st = thip(t, hipMemcpyAsync(t->ws + t->L.P, w, nb, hipMemcpyHostToDevice, t->stream),
                   "weights")))
        return st;
    if ((st = thip(t, hipMemsetAsync(t->ws + t->L.M, 0, nb, t->stream), "moments"))) return st;
    if ((st = thip(t, hipMemsetAsync(t->ws + t->L.V, 0, nb, t->stream), "moments"))) return st;
    if ((st = pack(t))) return st;
    if ((st = thip(t, hipStreamSynchronize(t->stream), "weights"))) return st;
    t->t = 0;
    t->have_w = true;
    return LBFD_OK;
}

lbfd_status lbfd_trainer_gradient(lbfd_trainer* t, const float* x, const float* y, int32_t n,
                                  const int32_t* idx, float* grad, double* loss) {
    if (!t) return LBFD_E_INVAL;
    lbfd_status st = batch_args(t, x, y, n, idx);
    if (st) return st;
    if ((st = forward_backward(t, x, y, n, idx))) return st;
    if (grad && (st = thip(t, hipMemcpyAsync(grad, t->ws + t->L.G, (size_t)t->np * 4,
                                             hipMemcpyDeviceToHost, t->stream), "gradient")))
        return st;
    if (loss && (st = thip(t, hipMemcpyAsync(loss, t->ws + t->L.loss, 8, hipMemcpyDeviceToHost,
                                             t->stream), "loss")))
        return st;
    return thip(t, hipStreamSynchronize(t->stream), "gradient");
}

lbfd_status lbfd_trainer_step(lbfd_trainer* t, const float* x, const float* y, int32_t n,
                              const int32_t* idx, float lr, double* loss) {
    if (!t) return LBFD_E_INVAL;
    if (!(lr > 0.f)) return tfail(t, LBFD_E_INVAL, "learning rate must be positive");
    lbfd_status st = batch_args(t, x, y, n, idx);
    if (st) return st;
    if ((st = forward_backward(t, x, y, n, idx))) return st;
    t->t += 1;
    const double c1 = 1.0 / (1.0 - std::pow((double)t->cfg.beta1, (double)t->t));
    const double c2 = 1.0 / (1.0 - std::pow((double)t->cfg.beta2, (double)t->t));
    hipLaunchKernelGGL(adam_kernel, dim3((t->np + TB - 1) / TB), dim3(TB), 0, t->stream,
                       tp<float>(t, t->L.P), tp<float>(t, t->L.M), tp<float>(t, t->L.V),
                       tp<float>(t, t->L.G), t->np, lr, t->cfg.beta1, t->cfg.beta2, t->cfg.eps,
                       (float)c1, (float)c2);
    if ((st = thip(t, hipGetLastError(), "adam"))) return st;
    if ((st = pack(t))) return st;
    if (loss) {
        if ((st = thip(t, hipMemcpyAsync(loss, t->ws + t->L.loss, 8, hipMemcpyDeviceToHost,
                                         t->stream), "loss")))
            return st;
        return thip(t, hipStreamSynchronize(t->stream), "loss");
    }
    return LBFD_OK;
}

lbfd_status lbfd_trainer_export(lbfd_trainer* t, float* w, float* norm, float* env) {
    if (!t) return LBFD_E_INVAL;
    lbfd_status st = thip(t, hipSetDevice(t->device), "hipSetDevice");
    if (st) return st;
    if (w && (st = thip(t, hipMemcpyAsync(w, t->ws + t->L.P, (size_t)t->np * 4,
                                          hipMemcpyDeviceToHost, t->stream), "export")))
        return st;
    TrainNorm nm;
    if ((st = thip(t, hipMemcpyAsync(&nm, t->ws + t->L.norm, sizeof(nm), hipMemcpyDeviceToHost,
                                     t->stream), "export")))
        return st;
    if ((st = thip(t, hipStreamSynchronize(t->stream), "export"))) return st;
    norm_to_host(nm, t->ni, t->no, norm, env);
    return LBFD_OK;
}

lbfd_status lbfd_fit_norm_noalloc(int32_t n_species, const float* x, const float* y, int32_t n,
                                  float* norm, float* envelope, void* hip_stream) {
    if (n_species < 1 || 2 + n_species > MLP_KIN || n_species > MLP_OUT)
        return LBFD_E_UNSUPPORTED;  // the staging block holds 16 inputs and 16 outputs
    if (!x || !y || n < 2 || (!norm && !envelope)) return LBFD_E_INVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LBFD_E_DEVICE;
    hipError_t e;
    TrainNorm* d = static_cast<TrainNorm*>(scratch_for_device(dev, &e));
    if (!d) return LBFD_E_DEVICE;
    const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int ni = 2 + n_species, no = n_species;
    // every field the outputs use is written by the kernel (one workgroup per
    // column), so nothing from an earlier call survives into this one
    hipLaunchKernelGGL(norm_fit_kernel, dim3(ni + no), dim3(TB), 0, s, x, y, n, ni, no, d);
    if (hipGetLastError() != hipSuccess) return LBFD_E_DEVICE;
    TrainNorm nm;
    if (hipMemcpyAsync(&nm, d, sizeof(nm), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LBFD_E_DEVICE;
    norm_to_host(nm, ni, no, norm, envelope);
    return LBFD_OK;
}

lbfd_status lbfd_trainer_destroy(lbfd_trainer* t) {
    delete t;
    return LBFD_OK;
}

const char* lbfd_trainer_last_error(const lbfd_trainer* t) {
    return t ? t->err.c_str() : "null trainer";
}

}  // extern "C"
