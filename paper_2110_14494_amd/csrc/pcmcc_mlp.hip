// Coefficient surrogate: a 1 -> 64 -> 64 -> 6 perceptron (tanh hidden
// layers) that maps standardised ln(E/N) to standardised log swarm
// coefficients (the inputs of the fluid model of arXiv:2110.14494 Sec. 2.2,
// computed by the swarms of Sec. 2.2.2).
//
//  * training (FP32): forward and backward over 64-point tiles held in LDS,
//    gradients reduced in a fixed order (bit-reproducible), full-batch Adam
//    with a cosine learning rate; one cooperative launch runs every epoch;
//  * inference (BF16 weights and activations, FP32 accumulation): the 64x64
//    layer and the output layer run on MFMA (v_mfma_f32_32x32x16_bf16); the
//    first layer is computed per lane straight into the MFMA operand layout;
//    a hidden activation is carried as s = (1 + tanh z) / 2, the logistic
//    function of 2 z, which the next layer absorbs into its bias;
//    the outputs flagged for a point's E/N cell fall back to interpolation
//    of the swarm table.
// Parameter vector (4678 floats): W1[64,1], b1[64], W2[64,64], b2[64],
// W3[6,64], b3[6], row-major.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "pcmcc_internal.hpp"

namespace cg = cooperative_groups;

namespace pcmcc {

constexpr int kH = 64, kOut = 6, kTile = 64;
constexpr unsigned kAllOut = (1u << kOut) - 1u;  // fallback mask with every output
constexpr int OFF_W1 = 0, OFF_B1 = 64, OFF_W2 = 128, OFF_B2 = 128 + 4096, OFF_W3 = OFF_B2 + 64,
              OFF_B3 = OFF_W3 + 384;
static_assert(OFF_B3 + 6 == kMlpParams, "parameter packing");

// ---------------------------------------------------------------------------
// Training: one tile of 64 points through forward and backward.  Gradients
// of W2 stay in registers (16 per thread, thread t owns row t/4, columns
// 16 (t%4) .. +15); the other 582 gradients live in LDS, each owned by one
// thread.  Everything is in a fixed order, so results are reproducible.
struct MlpLds {
  float P[kMlpParams];
  float H1[kTile][kH + 1];
  float H2[kTile][kH + 1];
  float D2[kTile][kH + 1];
  float x[kTile];
  float dy[kTile][kOut];
  float gsmall[kMlpParams - 4096];  // gradients of W1, b1, b2, W3, b3 (index = param - 4096 past OFF_W2)
  float loss[256];
};

// Index of a non-W2 parameter in gsmall.
__device__ __forceinline__ int small_idx(int param) { return param < OFF_W2 ? param : param - 4096; }

__device__ void tile_grad(MlpLds& L, const float* __restrict__ x, const float* __restrict__ t,
                          const float* __restrict__ m, int64_t n, int64_t p0, float inv_cnt, float gW2[16],
                          float& loss_acc) {
  const int tid = threadIdx.x;
  if (tid < kTile) L.x[tid] = (p0 + tid < n) ? x[p0 + tid] : 0.0f;
  __syncthreads();
  // h1 = tanh(W1 x + b1)
  for (int e = tid; e < kTile * kH; e += 256) {
    const int p = e >> 6, k = e & 63;
    L.H1[p][k] = tanhf(fmaf(L.P[OFF_W1 + k], L.x[p], L.P[OFF_B1 + k]));
  }
  __syncthreads();
  // h2 = tanh(W2 h1 + b2)
  for (int e = tid; e < kTile * kH; e += 256) {
    const int p = e >> 6, j = e & 63;
    float a = L.P[OFF_B2 + j];
    const float* w = &L.P[OFF_W2 + j * kH];
    for (int k = 0; k < kH; ++k) a = fmaf(w[k], L.H1[p][k], a);
    L.H2[p][j] = tanhf(a);
  }
  __syncthreads();
  // y = W3 h2 + b3; masked residual; dL/dy
  for (int e = tid; e < kTile * kOut; e += 256) {
    const int p = e / kOut, o = e % kOut;
    const int64_t q = p0 + p;
    float a = L.P[OFF_B3 + o];
    for (int j = 0; j < kH; ++j) a = fmaf(L.P[OFF_W3 + o * kH + j], L.H2[p][j], a);
    float r = 0.0f;
    if (q < n) r = m[q * kOut + o] * (a - t[q * kOut + o]);
    loss_acc = fmaf(r, r, loss_acc);
    L.dy[p][o] = 2.0f * r * inv_cnt;
  }
  __syncthreads();
  // dW3, db3
  for (int e = tid; e < kOut * kH + kOut; e += 256) {
    float g = 0.0f;
    if (e < kOut * kH) {
      const int o = e / kH, j = e % kH;
      for (int p = 0; p < kTile; ++p) g = fmaf(L.dy[p][o], L.H2[p][j], g);
    } else {
      const int o = e - kOut * kH;
      for (int p = 0; p < kTile; ++p) g += L.dy[p][o];
    }
    L.gsmall[small_idx(OFF_W3 + e)] += g;
  }
  // dz2 = (W3^T dy) (1 - h2^2)
  for (int e = tid; e < kTile * kH; e += 256) {
    const int p = e >> 6, j = e & 63;
    float a = 0.0f;
    for (int o = 0; o < kOut; ++o) a = fmaf(L.P[OFF_W3 + o * kH + j], L.dy[p][o], a);
    const float h = L.H2[p][j];
    L.D2[p][j] = a * ((1.0f - h) * (1.0f + h));
  }
  __syncthreads();
  // dW2 (registers), db2
  {
    const int j = tid >> 2, k0 = (tid & 3) * 16;
    for (int p = 0; p < kTile; ++p) {
      const float d = L.D2[p][j];
#pragma unroll
      for (int c = 0; c < 16; ++c) gW2[c] = fmaf(d, L.H1[p][k0 + c], gW2[c]);
    }
  }
  if (tid < kH) {
    float g = 0.0f;
    for (int p = 0; p < kTile; ++p) g += L.D2[p][tid];
    L.gsmall[small_idx(OFF_B2 + tid)] += g;
  }
  // dz1 = (W2^T dz2) (1 - h1^2), overwriting H1's slot would race with dW2: use H2's space
  __syncthreads();
  for (int e = tid; e < kTile * kH; e += 256) {
    const int p = e >> 6, k = e & 63;
    float a = 0.0f;
    for (int j = 0; j < kH; ++j) a = fmaf(L.P[OFF_W2 + j * kH + k], L.D2[p][j], a);
    const float h = L.H1[p][k];
    L.H2[p][k] = a * ((1.0f - h) * (1.0f + h));
  }
  __syncthreads();
  // dW1, db1
  if (tid < 2 * kH) {
    const int k = tid & 63;
    float g = 0.0f;
    if (tid < kH)
      for (int p = 0; p < kTile; ++p) g = fmaf(L.H2[p][k], L.x[p], g);
    else
      for (int p = 0; p < kTile; ++p) g += L.H2[p][k];
    L.gsmall[small_idx((tid < kH ? OFF_W1 : OFF_B1) + k)] += g;
  }
  __syncthreads();
}

// Gradient of the whole data set for the parameters in L.P: blocks take
// tiles b, b + G, ...; per-block partial gradients go to partial[b][*] and
// partial losses to ploss[b].
__device__ void block_grad(MlpLds& L, const MlpArgs& A, float* __restrict__ partial, float* __restrict__ ploss) {
  const int tid = threadIdx.x;
  float gW2[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) gW2[c] = 0.0f;
  for (int i = tid; i < kMlpParams - 4096; i += 256) L.gsmall[i] = 0.0f;
  float loss_acc = 0.0f;
  __syncthreads();
  const int64_t n_tiles = (A.n + kTile - 1) / kTile;
  for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x)
    tile_grad(L, A.x, A.t, A.mask, A.n, tl * kTile, A.inv_cnt, gW2, loss_acc);
  float* out = partial + (size_t)blockIdx.x * kMlpParams;
  const int j = tid >> 2, k0 = (tid & 3) * 16;
#pragma unroll
  for (int c = 0; c < 16; ++c) out[OFF_W2 + j * kH + k0 + c] = gW2[c];
  for (int i = tid; i < kMlpParams - 4096; i += 256) out[i < OFF_W2 ? i : i + 4096] = L.gsmall[i];
  L.loss[tid] = loss_acc;
  __syncthreads();
  if (tid == 0) {
    float s = 0.0f;
    for (int i = 0; i < 256; ++i) s += L.loss[i];
    ploss[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void k_mlp_grad(MlpArgs A) {
  extern __shared__ float smem[];
  MlpLds& L = *reinterpret_cast<MlpLds*>(smem);
  for (int i = threadIdx.x; i < kMlpParams; i += 256) L.P[i] = A.params[i];
  __syncthreads();
  block_grad(L, A, A.partial, A.ploss);
}

// Fixed-order reduction of the per-block partials.
__global__ void k_mlp_reduce(const float* __restrict__ partial, const float* __restrict__ ploss, int nb,
                             float* __restrict__ grad, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) {
    float s = 0.0f;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * kMlpParams + i];
    grad[i] = s;
  }
  if (i == 0) {
    float s = 0.0f;
    for (int b = 0; b < nb; ++b) s += ploss[b];
    *loss = s;
  }
}

// Every epoch: gradient (all blocks), fixed-order reduction and Adam update
// (one parameter per thread of the grid), then the blocks reload the
// parameters.  Two grid barriers per epoch.
__global__ __launch_bounds__(256) void k_mlp_train(MlpArgs A) {
  extern __shared__ float smem[];
  MlpLds& L = *reinterpret_cast<MlpLds*>(smem);
  cg::grid_group grid = cg::this_grid();
  const int gtid = blockIdx.x * 256 + threadIdx.x;
  const int nthr = gridDim.x * 256;
  for (int e = 0; e < A.epochs; ++e) {
    for (int i = threadIdx.x; i < kMlpParams; i += 256) L.P[i] = __hip_atomic_load(
        &A.params[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    block_grad(L, A, A.partial, A.ploss);
    grid.sync();
    const float lr = (float)(A.lr_min + 0.5 * (A.lr0 - A.lr_min) * (1.0 + cos(3.14159265358979323846 * e / A.epochs)));
    const float c1 = 1.0f / (1.0f - powf(A.beta1, (float)(e + 1)));
    const float c2 = 1.0f / (1.0f - powf(A.beta2, (float)(e + 1)));
    for (int i = gtid; i < kMlpParams; i += nthr) {
      float g = 0.0f;
      for (int b = 0; b < (int)gridDim.x; ++b) g += A.partial[(size_t)b * kMlpParams + i];
      const float m = A.beta1 * A.m[i] + (1.0f - A.beta1) * g;
      const float v = A.beta2 * A.v[i] + (1.0f - A.beta2) * g * g;
      A.m[i] = m;
      A.v[i] = v;
      A.params[i] -= lr * (m * c1) / (sqrtf(v * c2) + A.eps);
    }
    if (gtid == 0 && A.loss_hist) {
      float s = 0.0f;
      for (int b = 0; b < (int)gridDim.x; ++b) s += A.ploss[b];
      A.loss_hist[e] = s * A.inv_cnt;
    }
    grid.sync();
  }
}

// ---------------------------------------------------------------------------
// Inference.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

// Logistic function of t, with t given as -t log2(e) (the factor lives in the
// weights and biases that produce it): 1 / (1 + 2^-t log2 e), one exponential
// and one reciprocal; 0 and 1 at the ends.
__device__ __forceinline__ float logistic_l2(float neg_t_log2e) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(neg_t_log2e));
}

// The hidden layers use tanh(z) = 2 s - 1 with s = logistic(2 z): the next
// layer takes s as its input, with its weights doubled (exact in bfloat16, so
// the matrix operands are the weights themselves and the doubling is applied
// to the product) and its bias reduced by the row sum of its bfloat16 weights.
// Each activation is then one multiply-add, one exponential, one add and one
// reciprocal; s, not tanh(z), is what is rounded to bfloat16.
constexpr float kM2L2E = -2.0f * 1.4426950408889634f;  // -2 log2(e)

constexpr int kMaskLds = 4096;

// Operand fragments in LDS: for MFMA k-step s and lane l, 8 bf16 values.
struct InferLds {
  bf16x8 A2[2][4][64];  // W2: M-block m (output features 32m..), k-step s (inputs 16s + 8 (l/32) + q)
  bf16x8 A3[4][64];     // W3 padded to 32 rows; k-step s, q -> feature 32 (s/2) + 8 (2 (s%2) + q/4) + 4 (l/32) + q%4
  float a1[64], c1[64];  // layer 1: -2 log2(e) (W1, b1)
  float c2[64];          // layer 2: -2 log2(e) (b2 - row sums of bf16 W2)
  float y_scale[8], y_off[8];  // output: 2 sd_y, (b3 - row sums of bf16 W3) sd_y + mu_y
  uint8_t mask[kMaskLds];      // the fallback mask per cell, when it has at most kMaskLds cells
};

// The tiles of one wave, 32 points each: lanes l and l + 32 both work on
// point l of a tile (the two halves of the MFMA operands), and each writes its
// half of the outputs.  MASK_LDS: the fallback mask sits in LDS (otherwise it
// is read from global memory); the two cases are separate instantiations so
// that each read is a plain LDS or global load, never a generic one, whose wait
// would also wait for the field read ahead for the next tile.  The table rows
// of the outputs that fall back are read before the next tile's field and
// before the network, so that their latency overlaps the network and waiting
// for them does not wait for that prefetch.
template <bool MASK_LDS>
__device__ __forceinline__ void infer_tiles(const InferArgs& A, const InferLds& L, int lane, int64_t wave,
                                            int64_t nwave) {
  const int half = lane >> 5, col = lane & 31;
  const int64_t stride = nwave * 32;
  // the field of the lane's point in the wave's next tile, read one
  // iteration ahead (an index clamped into the array, so that the load needs
  // no branch)
  float en_next = A.EN[min(wave * 32 + col, A.n - 1)];
  for (int64_t p0 = wave * 32; p0 < A.n; p0 += stride) {
    const int64_t p = p0 + col;
    const bool valid = p < A.n;
    const float EN = valid ? en_next : 1.0f;
    const float lnEN = logf(EN);
    const float xs = (lnEN - A.mu_x) * A.inv_sd_x;
    // bit o set: output o of this point's cell takes the table
    unsigned fbm = 0u;
    float tf = 0.0f, ta[4] = {0.0f, 0.0f, 0.0f, 0.0f}, tb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (A.n_cells > 0) {
      const int cell = min(max((int)floorf((lnEN - A.cell_lo) * A.inv_cell_w), 0), A.n_cells - 1);
      fbm = (unsigned)(MASK_LDS ? L.mask[cell] : A.fb_mask[cell]) & kAllOut;
      if (fbm) {
        const float u = fminf(fmaxf((lnEN - A.tab_lo) * A.inv_tab_w, 0.0f), (float)(A.n_nodes - 1));
        const float fl = fminf(floorf(u), (float)(A.n_nodes - 2));
        tf = u - fl;
        // this lane's outputs 4 half + j of the nodes on either side
        const float* row = A.table + (size_t)(int)fl * kOut + 4 * half;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * half + j < kOut) {
            ta[j] = row[j];
            tb[j] = row[kOut + j];
          }
      }
    }
    en_next = A.EN[min(p + stride, A.n - 1)];
    floatx16 c3;
    for (int r = 0; r < 16; ++r) c3[r] = 0.0f;
    // The perceptron runs unless every output of every point of the wave
    // falls back to the table (the condition is wave-uniform, as the matrix
    // instructions need).
    if (__ballot(valid && fbm != kAllOut) != 0) {
      // layer 2: C2[m] = W2[32m.., :] s1 over 4 k-steps of 16
      floatx16 c2[2];
      for (int m = 0; m < 2; ++m)
        for (int r = 0; r < 16; ++r) c2[m][r] = 0.0f;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        bf16x8 b;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = 16 * s + 8 * half + q;
          b[q] = (__bf16)logistic_l2(fmaf(L.a1[k], xs, L.c1[k]));
        }
        c2[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.A2[0][s][lane], b, c2[0], 0, 0, 0);
        c2[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.A2[1][s][lane], b, c2[1], 0, 0, 0);
      }
      // activation of layer 2 (z = 2 C2 + b2 - row sum); rows of C2 held by
      // this lane: 8 i + 4 half + j (i = reg / 4, j = reg % 4)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int m = s >> 1;
        bf16x8 b;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int i = 2 * (s & 1) + (q >> 2), j = q & 3;
          const int row = 8 * i + 4 * half + j;
          b[q] = (__bf16)logistic_l2(fmaf(c2[m][4 * i + j], 2.0f * kM2L2E, L.c2[32 * m + row]));
        }
        c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.A3[s][lane], b, c3, 0, 0, 0);
      }
    }
    if (!valid) continue;
    // outputs: rows 4 half + j (j < 4) of C3 are outputs 0..3 (half 0) and 4..7 (half 1)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = 4 * half + j;
      if (o >= kOut) break;
      float y = fmaf(c3[j], L.y_scale[o], L.y_off[o]);
      if ((fbm >> o) & 1u) y = fmaf(tf, tb[j] - ta[j], ta[j]);
      A.out[(size_t)o * A.n + p] = y;
    }
  }
}

// Five waves per SIMD (92 registers, no spills): left to itself the compiler
// gives the table rows held across the network registers of their own (103)
// and the kernel would drop to four.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_mlp_infer(InferArgs A) {
  __shared__ InferLds L;
  const int tid = threadIdx.x;
  const float* P = A.params;
  for (int i = tid; i < 2 * 4 * 64; i += 256) {
    const int m = i >> 8, s = (i >> 6) & 3, l = i & 63;
    bf16x8 v;
    for (int q = 0; q < 8; ++q) {
      const int o = 32 * m + (l & 31), k = 16 * s + 8 * (l >> 5) + q;
      v[q] = (__bf16)P[OFF_W2 + o * kH + k];
    }
    L.A2[m][s][l] = v;
  }
  for (int i = tid; i < 4 * 64; i += 256) {
    const int s = i >> 6, l = i & 63;
    bf16x8 v;
    for (int q = 0; q < 8; ++q) {
      const int o = l & 31;
      const int f = 32 * (s >> 1) + 8 * (2 * (s & 1) + (q >> 2)) + 4 * (l >> 5) + (q & 3);
      v[q] = (__bf16)(o < kOut ? P[OFF_W3 + o * kH + f] : 0.0f);
    }
    L.A3[s][l] = v;
  }
  if (tid < 64) {
    L.a1[tid] = kM2L2E * P[OFF_W1 + tid];
    L.c1[tid] = kM2L2E * P[OFF_B1 + tid];
    // the row sum of the bfloat16 weights in a fixed order (exact in double)
    double rs = 0.0;
    for (int k = 0; k < kH; ++k) rs += (double)(float)(__bf16)P[OFF_W2 + tid * kH + k];
    L.c2[tid] = kM2L2E * (float)((double)P[OFF_B2 + tid] - rs);
  }
  if (tid < 8) {
    double rs = 0.0;
    if (tid < kOut)
      for (int j = 0; j < kH; ++j) rs += (double)(float)(__bf16)P[OFF_W3 + tid * kH + j];
    L.y_scale[tid] = tid < kOut ? 2.0f * A.sd_y[tid] : 0.0f;
    L.y_off[tid] = tid < kOut ? (float)(((double)P[OFF_B3 + tid] - rs) * A.sd_y[tid] + A.mu_y[tid]) : 0.0f;
  }
  const bool mask_lds = A.n_cells <= kMaskLds;
  if (mask_lds)
    for (int i = tid; i < A.n_cells; i += 256) L.mask[i] = A.fb_mask[i];
  __syncthreads();
  const int64_t wave = (int64_t)blockIdx.x * 4 + (tid >> 6);
  const int64_t nwave = (int64_t)gridDim.x * 4;
  if (mask_lds)
    infer_tiles<true>(A, L, tid & 63, wave, nwave);
  else
    infer_tiles<false>(A, L, tid & 63, wave, nwave);
}

// ---------------------------------------------------------------------------
size_t mlp_lds_bytes() { return sizeof(MlpLds); }

hipError_t launch_mlp_grad(const MlpArgs& a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(256), sizeof(MlpLds), stream, a);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float* partial, const float* ploss, int nb, float* grad, float* loss,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, partial, ploss, nb, grad,
                     loss);
  return hipGetLastError();
}

hipError_t occupancy_mlp_train(int* blocks_per_cu) {
  return coresident_blocks((const void*)k_mlp_train, 256, sizeof(MlpLds), blocks_per_cu);
}

hipError_t launch_mlp_train(const MlpArgs& a, int grid, hipStream_t stream) {
  void* kargs[] = {(void*)&a};
  return hipLaunchCooperativeKernel((const void*)k_mlp_train, dim3(grid), dim3(256), kargs, sizeof(MlpLds), stream);
}

hipError_t launch_mlp_infer(const InferArgs& a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace pcmcc
