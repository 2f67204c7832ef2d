// Coefficient network of the solver (Sec. 3.1, Fig. 4): alpha_hat = alpha_0 +
// s_out f_theta(s_in Re/Im alpha_0), Adam on theta (Sec. 3.3).  One network per
// reconstruction, shared by its N_i incidences: each incidence is a row of
// width D = 2 K^2 ([Re alpha_0[i, :], Im alpha_0[i, :]]), layers D -> H -> H
// -> D with tanh after the first two.  Parameters of one reconstruction are
// flat: per layer a block of (in + 1) x out values, row-major [k][n], the last
// row the bias.
//
// The three products of a layer are skinny GEMMs with per-reconstruction
// weights (N_i <= 64 rows): each weight is used by N_i rows only, so the
// weight stream from HBM and the Adam state dominate.  One workgroup computes
// all rows of 64 output columns, staging 64 reduction indices of the rows and
// the matching weight tile through LDS: in FP32 on the matrix cores (below,
// k_fc_*_mfma), in FP64 on the vector units with each wave owning a quarter
// of the rows (k_fc_fwd, k_fc_bwd).  The weight gradients and Adam are one
// kernel over all layers (k_fc_adam).
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include "cplx.h"

namespace pdfk {

constexpr int kFcCols = 64;    // output columns per workgroup (one per lane)
constexpr int kFcRed = 64;     // reduction indices staged per pass
constexpr int kFcMaxRows = 64; // incidences per reconstruction
constexpr int kFcAdamRows = 64;  // weight rows per Adam tile (16 per wave)

template <typename T>
__device__ __forceinline__ T fc_tanh(T z);
template <>
__device__ __forceinline__ float fc_tanh<float>(float z) { return tanhf(z); }
template <>
__device__ __forceinline__ double fc_tanh<double>(double z) { return tanh(z); }

// Row r, column c of a real row matrix given either as T [rows][width] or as
// the [Re | Im] split of complex [rows][Q] values (width 2Q) times `scale`.
template <typename T>
struct FcRows {
  const T* re = nullptr;        // real rows, or null
  const cx<T>* cxv = nullptr;   // complex rows (split), or null
  int width = 0;                // real width (2Q for complex rows)
  T scale = T(1);               // factor on complex rows
  __device__ __forceinline__ T at(int r, int c) const {
    if (cxv) {
      const int q = width >> 1;
      const cx<T> z = cxv[r * q + (c < q ? c : c - q)];
      return scale * (c < q ? z.x : z.y);
    }
    return re[r * width + c];
  }
};

template <typename T>
struct FcLayerArgs {
  FcRows<T> in;          // per reconstruction: rows [R][in]; .re/.cxv point at reconstruction 0
  size_t in_stride;      // elements (T or cx<T>) between reconstructions
  const T* theta;        // parameters of reconstruction 0, this layer's block
  size_t theta_stride;   // parameters per reconstruction
  int R, n_in, n_out;    // rows, layer input and output widths
  // forward epilogue: hidden (tanh) rows into act; the output layer writes its plain rows
  // into act (FP32, joined to alpha_hat by k_fc_join) or alpha_0 + out_scale times them
  // into alpha_hat (FP64)
  T* act;                // [B][R][n_out] or null
  T out_scale;
  const cx<T>* alpha0;   // [B][R][Q] (output layer)
  cx<T>* alpha_hat;      // [B][R][Q] (output layer)
  // input-gradient epilogue: gprev = (sum_c g[r][c] W[n][c]) (1 - a[r][n]^2)
  const T* a_prev;       // [B][R][n_in]
  T* gprev;              // [B][R][n_in]
};

constexpr int kFcThreads = 256;
constexpr int kFcWTile = kFcRed * kFcCols / kFcThreads;   // weight-tile values per thread

// out[r][n] = sum_c A[r][c] W'(c, n) for the 64 columns n0.. of this workgroup,
// with W'(c, n) = W[c][n] (forward, TRANS = false) or W[n][c] (input gradient).
// The rows (at most 4 RPW) and the weight tile of reduction block c + 1 are
// loaded into registers while block c is multiplied out of LDS.
template <typename T, int RPW, bool TRANS>
__device__ __forceinline__ void fc_gemm_tile(T* As, T* Ws, const FcRows<T>& in, const T* W, int R, int n_red,
                                             int ld_w, int n_cols, int n0, T (&acc)[RPW]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T wr[kFcWTile], ar[RPW];
  auto load = [&](int c0) {
#pragma unroll
    for (int i = 0; i < kFcWTile; ++i) {
      const int e = threadIdx.x + i * kFcThreads;
      if (!TRANS) {   // W[c][n]: consecutive threads along n
        const int c = c0 + e / kFcCols, n = n0 + e % kFcCols;
        wr[i] = (c < n_red && n < n_cols) ? W[c * ld_w + n] : T(0);
      } else {        // W[n][c]: consecutive threads along c
        const int n = n0 + e / kFcRed, c = c0 + e % kFcRed;
        wr[i] = (c < n_red && n < n_cols) ? W[n * ld_w + c] : T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int e = threadIdx.x + i * kFcThreads, r = e / kFcRed, c = c0 + e % kFcRed;
      ar[i] = (r < R && c < n_red) ? in.at(r, c) : T(0);
    }
  };
#pragma unroll
  for (int i = 0; i < RPW; ++i) acc[i] = T(0);
  load(0);
  for (int c0 = 0; c0 < n_red; c0 += kFcRed) {
#pragma unroll
    for (int i = 0; i < kFcWTile; ++i) {
      const int e = threadIdx.x + i * kFcThreads;
      if (!TRANS) Ws[(e / kFcCols) * (kFcCols + 1) + e % kFcCols] = wr[i];
      else Ws[(e % kFcRed) * (kFcCols + 1) + e / kFcRed] = wr[i];   // transposed into Ws[c][n]
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) As[threadIdx.x + i * kFcThreads] = ar[i];
    __syncthreads();
    if (c0 + kFcRed < n_red) load(c0 + kFcRed);
    const T* arow = As + wv * RPW * kFcRed;
#pragma unroll 4
    for (int cc = 0; cc < kFcRed; ++cc) {
      const T w = Ws[cc * (kFcCols + 1) + lane];
#pragma unroll
      for (int i = 0; i < RPW; ++i) acc[i] += arow[i * kFcRed + cc] * w;
    }
    __syncthreads();
  }
}

// Forward of one layer.  Grid (ceil(n_out / 64), B), 256 threads; R <= 4 RPW.
template <typename T, int RPW, bool OUT>
__global__ void __launch_bounds__(256) k_fc_fwd(FcLayerArgs<T> a) {
  extern __shared__ unsigned char fc_smem[];
  T* As = reinterpret_cast<T*>(fc_smem);
  T* Ws = As + kFcMaxRows * kFcRed;
  const int b = blockIdx.y, n0 = blockIdx.x * kFcCols;
  FcRows<T> in = a.in;
  if (in.cxv) in.cxv += size_t(b) * a.in_stride; else in.re += size_t(b) * a.in_stride;
  const T* W = a.theta + size_t(b) * a.theta_stride;
  T acc[RPW];
  fc_gemm_tile<T, RPW, false>(As, Ws, in, W, a.R, a.n_in, a.n_out, a.n_out, n0, acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n = n0 + lane;
  if (n >= a.n_out) return;
  const T bias = W[size_t(a.n_in) * a.n_out + n];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = wv * RPW + i;
    if (r >= a.R) break;
    const T z = acc[i] + bias;
    const size_t row = size_t(b) * a.R + r;
    if (!OUT) {
      a.act[row * a.n_out + n] = fc_tanh(z);
    } else {   // Delta alpha row [Re | Im] added to alpha_0
      const int q = a.n_out >> 1, mode = n < q ? n : n - q;
      const T* a0 = reinterpret_cast<const T*>(a.alpha0 + row * q + mode);
      T* ah = reinterpret_cast<T*>(a.alpha_hat + row * q + mode);
      const int part = n < q ? 0 : 1;
      ah[part] = a0[part] + a.out_scale * z;
    }
  }
}

// Gradient with respect to a hidden layer's pre-activation:
// gprev[r][n] = (sum_c g[r][c] W[n][c]) (1 - a_prev[r][n]^2), n < n_in.
// Grid (ceil(n_in / 64), B), 256 threads.
template <typename T, int RPW>
__global__ void __launch_bounds__(256) k_fc_bwd(FcLayerArgs<T> a) {
  extern __shared__ unsigned char fc_smem[];
  T* As = reinterpret_cast<T*>(fc_smem);
  T* Ws = As + kFcMaxRows * kFcRed;
  const int b = blockIdx.y, n0 = blockIdx.x * kFcCols;
  FcRows<T> g = a.in;
  if (g.cxv) g.cxv += size_t(b) * a.in_stride; else g.re += size_t(b) * a.in_stride;
  const T* W = a.theta + size_t(b) * a.theta_stride;
  T acc[RPW];
  fc_gemm_tile<T, RPW, true>(As, Ws, g, W, a.R, a.n_out, a.n_out, a.n_in, n0, acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n = n0 + lane;
  if (n >= a.n_in) return;
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = wv * RPW + i;
    if (r >= a.R) break;
    const size_t idx = (size_t(b) * a.R + r) * a.n_in + n;
    const T av = a.a_prev[idx];
    a.gprev[idx] = acc[i] * (T(1) - av * av);
  }
}

// ---- FP32 layer products on the matrix cores (v_mfma_f32_32x32x2f32)
//
// Same tiles and staging as above: rows (RT tiles of 32) x 64 output columns per
// workgroup, reduction blocks of 64 staged through LDS (rows at a padded stride
// of 65 floats, so the 32 lanes reading one reduction index hit 32 banks).  Wave
// w multiplies column tile (w & 1) over half (w >> 1) of each block; the two
// halves are summed through LDS at the end.  Operand layout of the 32x32x2
// product: lane l supplies A[l mod 32][l / 32] and B[l / 32][l mod 32]; register
// j of lane l holds D[(j & 3) + 8 (j >> 2) + 4 (l / 32)][l mod 32].
typedef float fc_floatx16 __attribute__((ext_vector_type(16)));
constexpr int kFcLdA = kFcRed + 1;
constexpr size_t kFcMfmaLds = sizeof(float) * (size_t(kFcMaxRows) * kFcLdA + size_t(kFcRed) * (kFcCols + 1));

template <int RT, bool TRANS>
__device__ __forceinline__ void fc_gemm_tile_mfma(float* As, float* Ws, const FcRows<float>& in, const float* W, int R,
                                                  int n_red, int ld_w, int n_cols, int n0, fc_floatx16 (&acc)[RT]) {
  constexpr int NA = RT * 32 * kFcRed / kFcThreads;   // staged row values per thread
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ct = wv & 1, kh = wv >> 1, l32 = lane & 31, lhi = lane >> 5;
  float wr[kFcWTile], ar[NA];
  auto load = [&](int c0) {
#pragma unroll
    for (int i = 0; i < kFcWTile; ++i) {
      const int e = threadIdx.x + i * kFcThreads;
      if (!TRANS) {
        const int c = c0 + e / kFcCols, n = n0 + e % kFcCols;
        wr[i] = (c < n_red && n < n_cols) ? W[c * ld_w + n] : 0.f;
      } else {
        const int n = n0 + e / kFcRed, c = c0 + e % kFcRed;
        wr[i] = (c < n_red && n < n_cols) ? W[n * ld_w + c] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = threadIdx.x + i * kFcThreads, r = e / kFcRed, c = c0 + e % kFcRed;
      ar[i] = (r < R && c < n_red) ? in.at(r, c) : 0.f;
    }
  };
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[t][j] = 0.f;
  load(0);
  for (int c0 = 0; c0 < n_red; c0 += kFcRed) {
#pragma unroll
    for (int i = 0; i < kFcWTile; ++i) {
      const int e = threadIdx.x + i * kFcThreads;
      if (!TRANS) Ws[(e / kFcCols) * (kFcCols + 1) + e % kFcCols] = wr[i];
      else Ws[(e % kFcRed) * (kFcCols + 1) + e / kFcRed] = wr[i];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = threadIdx.x + i * kFcThreads;
      As[(e / kFcRed) * kFcLdA + e % kFcRed] = ar[i];
    }
    __syncthreads();
    if (c0 + kFcRed < n_red) load(c0 + kFcRed);
#pragma unroll
    for (int kk = 0; kk < kFcRed / 4; ++kk) {
      if (c0 + kh * (kFcRed / 2) + 2 * kk >= n_red) break;   // wave-uniform: only zero padding is left
      const int c = kh * (kFcRed / 2) + 2 * kk + lhi;
      const float bv = Ws[c * (kFcCols + 1) + ct * 32 + l32];
#pragma unroll
      for (int t = 0; t < RT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(As[(t * 32 + l32) * kFcLdA + c], bv, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  // the second half's partial tiles into the first half's waves (As reused: 2 x RT x 1024 floats)
  float* red = As;
  if (kh == 1)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int j = 0; j < 16; ++j) red[((ct * RT + t) * 16 + j) * 64 + lane] = acc[t][j];
  __syncthreads();
  if (kh == 0)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] += red[((ct * RT + t) * 16 + j) * 64 + lane];
}

// Row and column of register j of this lane in the workgroup's output block.
__device__ __forceinline__ int fc_mfma_row(int t, int j) {
  return t * 32 + (j & 3) + 8 * (j >> 2) + 4 * ((threadIdx.x & 63) >> 5);
}
__device__ __forceinline__ int fc_mfma_col(int n0) { return n0 + ((threadIdx.x >> 6) & 1) * 32 + (threadIdx.x & 31); }

// Reconstruction b and column tile t of this workgroup in a one-dimensional grid of ntiles x B.
// Consecutive workgroups go to the eight XCDs in turn; with B a multiple of 8 the tiles of one
// reconstruction are given to workgroups of one XCD, so its staged rows are fetched into one L2.
__device__ __forceinline__ void fc_tile_of(int ntiles, int& b, int& t) {
  const int id = blockIdx.x, B = gridDim.x / ntiles;
  if (B % 8 == 0) {
    const int x = id & 7, sl = id >> 3;
    b = x + 8 * (sl / ntiles);
    t = sl % ntiles;
  } else {
    b = id / ntiles;
    t = id % ntiles;
  }
}

// Forward of one layer, FP32 on MFMA: tanh rows of a hidden layer, or the output layer's plain
// rows (OUT).  Grid ceil(n_out / 64) x B (one-dimensional, fc_tile_of), 256 threads; R <= 32 RT.
template <int RT, bool OUT>
__global__ void __launch_bounds__(256) k_fc_fwd_mfma(FcLayerArgs<float> a) {
  extern __shared__ unsigned char fc_smem[];
  float* As = reinterpret_cast<float*>(fc_smem);
  float* Ws = As + kFcMaxRows * kFcLdA;
  int b, tile;
  fc_tile_of((a.n_out + kFcCols - 1) / kFcCols, b, tile);
  const int n0 = tile * kFcCols;
  FcRows<float> in = a.in;
  if (in.cxv) in.cxv += size_t(b) * a.in_stride; else in.re += size_t(b) * a.in_stride;
  const float* W = a.theta + size_t(b) * a.theta_stride;
  fc_floatx16 acc[RT];
  fc_gemm_tile_mfma<RT, false>(As, Ws, in, W, a.R, a.n_in, a.n_out, a.n_out, n0, acc);
  if ((threadIdx.x >> 6) >= 2) return;
  const int n = fc_mfma_col(n0);
  if (n >= a.n_out) return;
  const float bias = W[size_t(a.n_in) * a.n_out + n];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int r = fc_mfma_row(t, j);
      if (r >= a.R) continue;
      const float z = acc[t][j] + bias;
      const size_t row = size_t(b) * a.R + r;
      a.act[row * a.n_out + n] = OUT ? z : fc_tanh(z);   // output rows: joined to alpha_hat by k_fc_join
    }
}

// Pre-activation gradient of a hidden layer, FP32 on MFMA.  Grid ceil(n_in / 64) x B
// (one-dimensional, fc_tile_of), 256 threads.
template <int RT>
__global__ void __launch_bounds__(256) k_fc_bwd_mfma(FcLayerArgs<float> a) {
  extern __shared__ unsigned char fc_smem[];
  float* As = reinterpret_cast<float*>(fc_smem);
  float* Ws = As + kFcMaxRows * kFcLdA;
  int b, tile;
  fc_tile_of((a.n_in + kFcCols - 1) / kFcCols, b, tile);
  const int n0 = tile * kFcCols;
  FcRows<float> g = a.in;
  if (g.cxv) g.cxv += size_t(b) * a.in_stride; else g.re += size_t(b) * a.in_stride;
  const float* W = a.theta + size_t(b) * a.theta_stride;
  fc_floatx16 acc[RT];
  fc_gemm_tile_mfma<RT, true>(As, Ws, g, W, a.R, a.n_out, a.n_out, a.n_in, n0, acc);
  if ((threadIdx.x >> 6) >= 2) return;
  const int n = fc_mfma_col(n0);
  if (n >= a.n_in) return;
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int r = fc_mfma_row(t, j);
      if (r >= a.R) continue;
      const size_t idx = (size_t(b) * a.R + r) * a.n_in + n;
      const float av = a.a_prev[idx];
      a.gprev[idx] = acc[t][j] * (1.f - av * av);
    }
}

// out[row] = scale [Re z[row][:], Im z[row][:]] for the rows of Q complex values (n = rows Q
// in all): the network's real rows of alpha_0 and of g, written once so that the layer
// kernels stage contiguous floats.  Grid ceil(n / 256).
template <typename T>
__global__ void __launch_bounds__(256) k_fc_split(const cx<T>* z, T scale, T* out, int Q, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t row = i / Q, c = i % Q;
  const cx<T> v = z[i];
  out[row * 2 * Q + c] = scale * v.x;
  out[row * 2 * Q + Q + c] = scale * v.y;
}

// alpha_hat[row] = alpha_0[row] + scale (y[row][:Q] + i y[row][Q:]) (n = rows Q values).
// Grid ceil(n / 256).
template <typename T>
__global__ void __launch_bounds__(256) k_fc_join(const cx<T>* alpha0, const T* y, T scale, cx<T>* alpha_hat, int Q,
                                                 size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t row = i / Q, c = i % Q;
  const cx<T> a = alpha0[i];
  const T re = y[row * 2 * Q + c], im = y[row * 2 * Q + Q + c];
  alpha_hat[i] = cx<T>{a.x + scale * re, a.y + scale * im};
}

template <typename T>
struct FcAdamArgs {
  FcRows<T> in[3];        // layer inputs of reconstruction 0: X (split alpha_0), A1, A2
  size_t in_stride[3];
  FcRows<T> g[3];         // gradients at the layer outputs: G1, G2, [Re g | Im g]
  size_t g_stride[3];
  int n_in[3], n_out[3];
  size_t off[3];          // parameter block offsets
  int tile_start[4];      // first tile of each layer (tile_start[3] = tiles per reconstruction)
  int R;
  int xcd_order;          // 1: the tiles of a reconstruction on one XCD (needs B % 8 == 0)
  T* theta;
  T* m;
  T* v;
  size_t theta_stride;
  double lr1, ic2;        // lr / (1 - b1^t), 1 / (1 - b2^t)
  double b1, b2, eps;
};

// Weight gradients dW[k][n] = sum_r in[r][k] g[r][n] (in[r][n_in] = 1: bias row)
// of every layer, each followed at once by its bias-corrected Adam update.
// Grid tiles per reconstruction x B (one-dimensional), 256 threads; a tile is 64 / V rows x
// 64 V columns of one layer's block, 16 / V rows per wave and V adjacent
// columns per lane (V = 2: every theta, m, v access moves two values, which
// halves the memory instructions; it needs even widths and block offsets), so
// each staged gradient tile serves 64 / V weight rows.  Each weight's sum runs
// over the rows in the same order for either V.
template <int V>
struct FcAdamTile {
  static constexpr int ROWS = kFcAdamRows / V, COLS = kFcCols * V, RW = ROWS / 4;
};

template <typename T, int V>
__global__ void __launch_bounds__(256) k_fc_adam(FcAdamArgs<T> a) {
  using Tl = FcAdamTile<V>;
  constexpr int ROWS = Tl::ROWS, COLS = Tl::COLS, RW = Tl::RW;
  __shared__ T Is[kFcMaxRows * ROWS];
  __shared__ T Gs[kFcMaxRows * COLS];
  // one-dimensional grid of tiles x B workgroups.  Consecutive workgroups go
  // to the eight XCDs in turn, each with its own L2; with B a multiple of 8
  // the tiles of one reconstruction are given to workgroups of one XCD, so its
  // staged rows are fetched into one L2 instead of eight
  const int tiles = a.tile_start[3];
  int b, tt;
  if (a.xcd_order) {
    const int id = blockIdx.x, x = id & 7, s = id >> 3;
    b = x + 8 * (s / tiles);
    tt = s % tiles;
  } else {
    b = blockIdx.x / tiles;
    tt = blockIdx.x % tiles;
  }
  int l = 0;
  while (l < 2 && tt >= a.tile_start[l + 1]) ++l;
  const int n_in = a.n_in[l], n_out = a.n_out[l];
  const int ntn = (n_out + COLS - 1) / COLS;
  const int t = tt - a.tile_start[l];
  const int k0 = (t / ntn) * ROWS, n0 = (t % ntn) * COLS;
  FcRows<T> in = a.in[l], g = a.g[l];
  if (in.cxv) in.cxv += size_t(b) * a.in_stride[l]; else in.re += size_t(b) * a.in_stride[l];
  if (g.cxv) g.cxv += size_t(b) * a.g_stride[l]; else g.re += size_t(b) * a.g_stride[l];
  const int R = a.R;
  constexpr int NI = kFcMaxRows * ROWS / kFcThreads, NG = kFcMaxRows * COLS / kFcThreads;
  T iv[NI], gv_[NG];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int e = threadIdx.x + i * kFcThreads, r = e / ROWS, k = k0 + e % ROWS;
    iv[i] = (r < R && k < n_in) ? in.at(r, k) : (k == n_in ? T(1) : T(0));
  }
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int e = threadIdx.x + i * kFcThreads, r = e / COLS, n = n0 + e % COLS;
    gv_[i] = (r < R && n < n_out) ? g.at(r, n) : T(0);
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int e = threadIdx.x + i * kFcThreads;
    if (e < R * ROWS) Is[e] = iv[i];
  }
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int e = threadIdx.x + i * kFcThreads;
    if (e < R * COLS) Gs[e] = gv_[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n = n0 + V * lane;
  if (n >= n_out) return;   // with V = 2 and an even width, n + 1 < n_out too
  const size_t base = size_t(b) * a.theta_stride + a.off[l];
  // every row's theta, m, v requested before the gradient is formed (their HBM
  // latency overlaps the LDS products) and before the first store (the three
  // arrays may not be proven disjoint, so loads after a store would wait for it)
  using VT = typename std::conditional<V == 2, typename std::conditional<sizeof(T) == 4, float2, double2>::type,
                                       T>::type;
  VT th[RW], mo[RW], ve[RW];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int k = k0 + wv * RW + i;
    const size_t idx = base + size_t(k) * n_out + n;
    if (k <= n_in) {
      th[i] = *reinterpret_cast<const VT*>(a.theta + idx);
      mo[i] = *reinterpret_cast<const VT*>(a.m + idx);
      ve[i] = *reinterpret_cast<const VT*>(a.v + idx);
    } else {
      th[i] = VT{};
      mo[i] = VT{};
      ve[i] = VT{};
    }
  }
  T acc[RW][V];
#pragma unroll
  for (int i = 0; i < RW; ++i)
#pragma unroll
    for (int c = 0; c < V; ++c) acc[i][c] = T(0);
  for (int r = 0; r < R; ++r) {
    T gv[V];
#pragma unroll
    for (int c = 0; c < V; ++c) gv[c] = Gs[r * COLS + V * lane + c];
    const T* irow = Is + r * ROWS + wv * RW;
#pragma unroll
    for (int i = 0; i < RW; ++i)
#pragma unroll
      for (int c = 0; c < V; ++c) acc[i][c] += irow[i] * gv[c];
  }
  const T b1 = T(a.b1), b2 = T(a.b2), lr1 = T(a.lr1), ic2 = T(a.ic2), eps = T(a.eps);
  auto upd = [&](T gw, T th0, T m0, T v0, T& th1, T& m1, T& v1) {
    m1 = b1 * m0 + (T(1) - b1) * gw;
    v1 = b2 * v0 + (T(1) - b2) * (gw * gw);
    th1 = th0 - lr1 * m1 / (sqrt(v1 * ic2) + eps);
  };
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int k = k0 + wv * RW + i;
    if (k > n_in) break;
    const size_t idx = base + size_t(k) * n_out + n;
    if constexpr (V == 2) {
      VT t1, m1, v1;
      upd(acc[i][0], th[i].x, mo[i].x, ve[i].x, t1.x, m1.x, v1.x);
      upd(acc[i][1], th[i].y, mo[i].y, ve[i].y, t1.y, m1.y, v1.y);
      *reinterpret_cast<VT*>(a.m + idx) = m1;
      *reinterpret_cast<VT*>(a.v + idx) = v1;
      *reinterpret_cast<VT*>(a.theta + idx) = t1;
    } else {
      T t1, m1, v1;
      upd(acc[i][0], th[i], mo[i], ve[i], t1, m1, v1);
      a.m[idx] = m1;
      a.v[idx] = v1;
      a.theta[idx] = t1;
    }
  }
}

}  // namespace pdfk
