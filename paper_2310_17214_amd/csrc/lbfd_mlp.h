// lbfd_mlp.h -- data layout of the chemistry surrogate (a perceptron
// n_in -> 256 -> 256 -> n_out with ReLU, BF16 operands on the matrix cores,
// FP32 accumulation).  Shared by the kernels and the host runtime, which packs
// the weights into the fragment order the kernels read.
//
// Matrix-core fragments (v_mfma_f32_32x32x16_bf16, wave64): a product
// C[32 x 32] += A[32 x 16] B[16 x 32] takes from lane l the eight K-values
// (l / 32, j = 0..7) of row l % 32 of A and of column l % 32 of B, and
// returns C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in accumulator r.  Any
// K order works as long as A and B use the same one, so every layer's K
// order is chosen to be the order in which the previous layer's accumulators
// already sit: a hidden tile's 16 accumulators become two K-chunks of the
// next layer without moving data between lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfd {

constexpr int MLP_H = 256;    // hidden width
constexpr int MLP_KIN = 16;   // input features, padded (T, p, Y_1..Y_ns)
constexpr int MLP_OUT = 16;   // outputs, padded (omega_1..omega_ns)
constexpr int MLP_HT = MLP_H / 32;     // hidden tiles of 32
constexpr int MLP_HC = MLP_H / 16;     // hidden K-chunks of 16

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Inference weights as the workgroup holds them in LDS.
struct alignas(16) SurWeights {
    bf16x8 w1[MLP_HT][64];            // layer 1: output tile, lane
    bf16x8 w2[MLP_HT][MLP_HC][64];    // layer 2: output tile, K-chunk, lane
    bf16x8 w3[MLP_HC][64];            // layer 3 (rows >= n_out are zero): K-chunk, lane
    float b1[MLP_H], b2[MLP_H], b3[32];
};
static_assert(sizeof(SurWeights) == 157824, "LDS image size");

// Standardisation, envelope and checks (read with scalar loads).
struct SurPar {
    int n_in, n_out, enabled, pad;
    float mu_x[MLP_KIN], inv_sd_x[MLP_KIN], lo[MLP_KIN], hi[MLP_KIN];
    float mu_y[MLP_OUT], sd_y[MLP_OUT];
    float p_in;        // the constant thermodynamic-pressure input
    float resid_tol;   // |sum w| / (sum |w| + sd_sum) above this -> exact fallback
    float pos_tol;     // Y_k + dt w_k / rho below this (after the update) -> exact fallback
    float sd_sum;      // sum_k sd_y[k]: the residual's scale floor
    float clip_tol;    // overdraw of a species beyond clip_tol * sd_y[k] -> exact fallback
    float pad3[3];
};

// K order of the first layer: lane half h holds input features 8h..8h+7.
__host__ __device__ inline int mlp_k1(int lane, int j) { return 8 * (lane / 32) + j; }
// K order of hidden chunk c (0, 1) of hidden tile m: the accumulators
// 8c..8c+7 of a lane in half h hold features 32m + 16c + 8(j/4) + 4h + j%4.
__host__ __device__ inline int mlp_kh(int m, int c, int lane, int j) {
    return 32 * m + 16 * c + 8 * (j / 4) + 4 * (lane / 32) + j % 4;
}

}  // namespace lbfd
