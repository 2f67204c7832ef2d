// Warm-start network (an addition to the method): a fully connected network
// with GELU between its affine layers, trained with mean squared error and
// Adam.  GEMM operands are bfloat16, accumulation, biases, activations'
// pre-images, gradients and the master weights FP32.
//
// GEMMs run on v_mfma_f32_32x32x16_bf16.  One kernel template serves the
// three products of a layer (forward, gradient of the input, gradient of the
// weights) through the layout of its operands: each operand is either
// K-contiguous (row-major with the reduction index inner) or MN-contiguous
// (reduction index outer).  A 128 x 128 output tile per 256-thread workgroup,
// K staged through LDS 32 at a time, each wave owning a 64 x 64 quarter as
// 2 x 2 MFMA tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/pdf.h"
#include "handle.h"

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

// float -> bfloat16 bits, round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ u16 f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return u16((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u16(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

constexpr int GK = 64, LDK = GK + 8;  // K step, padded LDS row (bf16)
constexpr size_t kMlpSplitFloats = size_t(16) << 20;  // split-K workspace (64 MB)

enum Epi { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_GELU_GRAD = 3 };

struct GemmArgs {
  const u16* A;   // element (m, k) at A[m * lda + k] (K-contiguous) or A[k * lda + m]
  const u16* B;   // element (n, k) at B[n * ldb + k] (K-contiguous) or B[k * ldb + n]
  int lda, ldb;
  int Mr, Nc, K;
  float out_scale;    // EPI_BIAS: the stored value is out_scale * (product + bias)
  // epilogue
  float* C;           // FP32 [Mr][ldc]
  int ldc;
  const float* bias;  // [Nc]
  const float* zprev; // EPI_GELU_GRAD: pre-activation at (m, n), same layout as C
  u16* Cb;            // optional bfloat16 copy of the stored value, same layout as C
  // split K (products with few output tiles and a long K): workgroup z of the grid takes
  // K steps [z kchunk, (z + 1) kchunk) and writes its raw tile to part[z][Mr][Nc]; the
  // epilogue then runs in k_gemm_splitk_reduce over the parts in order.  kchunk = K: no split.
  int kchunk;
  float* part;
};

// The epilogue of output (m, n) with product v.
template <int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int m, int n, float v) {
  const size_t o = size_t(m) * g.ldc + n;
  if constexpr (EPI == EPI_BIAS_GELU) {
    v += g.bias[n];
    g.C[o] = v;
    g.Cb[o] = f2bf(gelu(v));
  } else if constexpr (EPI == EPI_BIAS) {
    g.C[o] = g.out_scale * (v + g.bias[n]);
  } else if constexpr (EPI == EPI_GELU_GRAD) {
    v *= gelu_grad(g.zprev[o]);
    g.C[o] = v;
    g.Cb[o] = f2bf(v);
  } else {
    g.C[o] = v;
  }
}

// An operand tile of GT rows (m or n) x GK k in flight: IT vectors of 8
// bfloat16 per thread, loaded from global memory (stage_load) into registers
// and later written to LDS as [row][k] (stage_store), so that the next K step's
// loads overlap the current step's products.
template <int GT>
struct StageRegs {
  static constexpr int IT = GT * GK / 8 / 256;
  uint4 v[IT];
};

__device__ __forceinline__ uint4 pack8(const u16 (&e)[8]) {
  return make_uint4(e[0] | (unsigned(e[1]) << 16), e[2] | (unsigned(e[3]) << 16), e[4] | (unsigned(e[5]) << 16),
                    e[6] | (unsigned(e[7]) << 16));
}

template <int GT, bool KCONTIG>
__device__ __forceinline__ void stage_load(StageRegs<GT>& R, const u16* src, int ld, int row0, int nrows, int k0,
                                           int K, int tid) {
  constexpr int IT = StageRegs<GT>::IT;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int v = tid + it * 256;
    if constexpr (KCONTIG) {  // GT rows x GK k: a vector is 8 consecutive k of one row
      const int r = v / (GK / 8), kq = (v % (GK / 8)) * 8;
      const int row = row0 + r, k = k0 + kq;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (row < nrows && k < K) {
        const u16* p = src + size_t(row) * ld + k;
        if (k + 8 <= K && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
          val = *reinterpret_cast<const uint4*>(p);
        } else {
          u16 e[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = (k + j < K) ? p[j] : u16(0);
          val = pack8(e);
        }
      }
      R.v[it] = val;
    } else {  // GK k-rows x GT rows: a vector is 8 consecutive rows of one k
      const int kk = v / (GT / 8), rq = (v % (GT / 8)) * 8;
      const int k = k0 + kk, row = row0 + rq;
      u16 e[8];
      if (k < K && row + 8 <= nrows) {
        const u16* p = src + size_t(k) * ld + row;
        if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
          R.v[it] = *reinterpret_cast<const uint4*>(p);
          continue;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = p[j];
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = (k < K && row + j < nrows) ? src[size_t(k) * ld + row + j] : u16(0);
      }
      R.v[it] = pack8(e);
    }
  }
}

template <int GT, bool KCONTIG>
__device__ __forceinline__ void stage_store(u16* S, const StageRegs<GT>& R, int tid) {
  constexpr int IT = StageRegs<GT>::IT;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int v = tid + it * 256;
    if constexpr (KCONTIG) {
      const int r = v / (GK / 8), kq = (v % (GK / 8)) * 8;
      *reinterpret_cast<uint4*>(S + r * LDK + kq) = R.v[it];
    } else {
      const int kk = v / (GT / 8), rq = (v % (GT / 8)) * 8;
      const uint4 val = R.v[it];
      const unsigned w[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
      for (int j = 0; j < 8; ++j) S[(rq + j) * LDK + kk] = u16(w[j >> 1] >> (16 * (j & 1)));
    }
  }
}

// GT x GT output tile per workgroup (GT = 128: each wave 2 x 2 MFMA tiles of
// 32 x 32; GT = 64: one tile each, for products too small to fill the chip
// with 128-wide tiles).  The next K step's operands are loaded into registers
// while the current step's products run.
template <int GT, bool AK, bool BK, int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  constexpr int WT = GT / 64;  // MFMA tiles per wave and dimension
  __shared__ __align__(16) u16 sA[GT * LDK];
  __shared__ __align__(16) u16 sB[GT * LDK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int wm = (w >> 1) * (GT / 2), wn = (w & 1) * (GT / 2);
  floatx16 acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);  // this workgroup's K range
  StageRegs<GT> ra, rb;
  stage_load<GT, AK>(ra, g.A, g.lda, m0, g.Mr, kb, ke, tid);
  stage_load<GT, BK>(rb, g.B, g.ldb, n0, g.Nc, kb, ke, tid);
  for (int k0 = kb; k0 < ke; k0 += GK) {
    stage_store<GT, AK>(sA, ra, tid);
    stage_store<GT, BK>(sB, rb, tid);
    __syncthreads();
    if (k0 + GK < ke) {
      stage_load<GT, AK>(ra, g.A, g.lda, m0, g.Mr, k0 + GK, ke, tid);
      stage_load<GT, BK>(rb, g.B, g.ldb, n0, g.Nc, k0 + GK, ke, tid);
    }
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      bf16x8 a[WT], b[WT];
#pragma unroll
      for (int i = 0; i < WT; ++i) {
        // lane (l % 32, l / 32) holds A[m = l % 32][k = 8 (l / 32) + j], likewise B[n][k]
        a[i] = *reinterpret_cast<const bf16x8*>(sA + (wm + 32 * i + (lane & 31)) * LDK + ks + 8 * (lane >> 5));
        b[i] = *reinterpret_cast<const bf16x8*>(sB + (wn + 32 * i + (lane & 31)) * LDK + ks + 8 * (lane >> 5));
      }
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[m][n]: lane l holds n = l % 32 and rows m = (r % 4) + 8 (r / 4) + 4 (l / 32)
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + 32 * i + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
        const int n = n0 + wn + 32 * j + (lane & 31);
        if (m >= g.Mr || n >= g.Nc) continue;
        if (gridDim.z > 1)
          g.part[(size_t(blockIdx.z) * g.Mr + m) * g.Nc + n] = acc[i][j][r];
        else
          gemm_epilogue<EPI>(g, m, n, acc[i][j][r]);
      }
}

// The split-K parts of each output added in order, then the epilogue.  Grid ceil(Mr Nc / 256).
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_splitk_reduce(GemmArgs g, int nsplit) {
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x, mn = size_t(g.Mr) * g.Nc;
  if (e >= mn) return;
  float v = 0.f;
  for (int z = 0; z < nsplit; ++z) v += g.part[z * mn + e];
  gemm_epilogue<EPI>(g, int(e / g.Nc), int(e % g.Nc), v);
}

// Input of the first layer: bfloat16 of s_in * x, rows gathered through idx.
// Row indices are clamped to [0, nrows) so that no index can address outside x.
__device__ __forceinline__ int clamp_row(const int* idx, int b, int nrows) {
  return idx ? min(max(idx[b], 0), nrows - 1) : b;
}

__global__ void k_input_bf16(const float* x, const int* idx, int nrows, float s_in, int B, int n, u16* out) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= size_t(B) * n) return;
  const int b = int(e / n), c = int(e % n);
  const int row = clamp_row(idx, b, nrows);
  out[e] = f2bf(s_in * x[size_t(row) * n + c]);
}

// MSE over [B][n]: dy = 2 (y - t) / (B n) (FP32 and bfloat16), per-row partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void k_mse(const float* y, const float* t, const int* idx, int nrows, int B,
                                             int n, float* dy, u16* dyb, double* rowsum) {
  __shared__ double red[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int row = clamp_row(idx, b, nrows);
  const float sc = 2.0f / (float(B) * float(n));
  double s = 0.0;
  for (int c = tid; c < n; c += 256) {
    const float d = y[size_t(b) * n + c] - t[size_t(row) * n + c];
    s += double(d) * d;
    const float g = sc * d;
    dy[size_t(b) * n + c] = g;
    dyb[size_t(b) * n + c] = f2bf(g);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) rowsum[b] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void k_mse_total(const double* rowsum, int B, int n, double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < B; ++b) s += rowsum[b];
  *loss = s / (double(B) * n);
}

// Bias gradient: column sums over the batch; 16 columns per workgroup, each
// summed by 16 threads (every 16th row) and the 16 parts added in a fixed
// order.  Grid ceil(n / 16), 256 threads.
__global__ __launch_bounds__(256) void k_colsum(const float* g, int B, int n, float* out) {
  constexpr int C = 16, S = 16;
  __shared__ float part[S][C];
  const int lc = threadIdx.x % C, sl = threadIdx.x / C, c = blockIdx.x * C + lc;
  float s = 0.f;
  if (c < n)
    for (int b = sl; b < B; b += S) s += g[size_t(b) * n + c];
  part[sl][lc] = s;
  __syncthreads();
  if (sl == 0 && c < n) {
    float t = 0.f;
    for (int k = 0; k < S; ++k) t += part[k][lc];
    out[c] = t;
  }
}

// Adam on FP32 master values; the bfloat16 copy follows.
__global__ void k_adam(float* w, const float* g, float* m, float* v, u16* wb, size_t n, float lr1, float b1,
                       float b2, float ic2, float eps) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr1 * mi / (sqrtf(vi * ic2) + eps);
  w[i] = wi;
  if (wb) wb[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float* x, u16* y, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

}  // namespace

struct pdf_mlp {
  int L = 0, bmax = 0;
  std::vector<int> sz;
  hipStream_t stream = nullptr;
  std::string err;
  int t = 0;  // Adam steps taken
  // per layer
  std::vector<float*> W, b, gW, gb, mW, vW, mb, vb;
  std::vector<u16*> Wb;
  // per layer activations: a[l] bfloat16 input [bmax][sz[l]], z[l] FP32 output [bmax][sz[l+1]]
  std::vector<u16*> a;
  std::vector<float*> z;
  float* dz[2] = {nullptr, nullptr};  // gradients of the pre-activations [bmax][max width], alternating
  u16* dzb[2] = {nullptr, nullptr};   // their bfloat16 copies
  double *rowsum = nullptr, *loss = nullptr;
  float* part = nullptr;  // split-K parts of the products [kMlpSplitFloats]
  std::vector<void*> owned;
};

namespace {

int mfail(pdf_mlp* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  pdf_set_global_error(msg);
  return code;
}

template <typename T>
int dalloc(pdf_mlp* n, T** p, size_t count) {
  if (hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
    return mfail(n, PDF_ENOMEM, "hipMalloc failed");
  n->owned.push_back(*p);
  return PDF_OK;
}

int mcheck(pdf_mlp* n, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(n, PDF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return PDF_OK;
}

// 128-wide tiles when they give at least two workgroups per CU, else 64-wide;
// with fewer than 512 tiles the K steps split over up to 16 workgroups per tile
// (at least four steps each, parts within the workspace) and a reduction
// applies the epilogue.
template <bool AK, bool BK, int EPI>
void launch_gemm(pdf_mlp* n, GemmArgs g) {
  const long big = long((g.Nc + 127) / 128) * ((g.Mr + 127) / 128);
  const long tiles = big >= 512 ? big : long((g.Nc + 63) / 64) * ((g.Mr + 63) / 64);
  const size_t mn = size_t(g.Mr) * g.Nc;
  int nsplit = 1;
  if (tiles < 512) {
    nsplit = int(std::min<long>(16, (1024 + tiles - 1) / tiles));
    nsplit = std::min(nsplit, std::max(1, g.K / (4 * GK)));
    nsplit = int(std::min<size_t>(size_t(nsplit), std::max<size_t>(1, kMlpSplitFloats / mn)));
  }
  g.kchunk = ((g.K + nsplit - 1) / nsplit + GK - 1) / GK * GK;
  nsplit = (g.K + g.kchunk - 1) / g.kchunk;
  g.part = n->part;
  if (big >= 512) {
    dim3 grid((g.Nc + 127) / 128, (g.Mr + 127) / 128, nsplit);
    hipLaunchKernelGGL((k_gemm_bf16<128, AK, BK, EPI>), grid, dim3(256), 0, n->stream, g);
  } else {
    dim3 grid((g.Nc + 63) / 64, (g.Mr + 63) / 64, nsplit);
    hipLaunchKernelGGL((k_gemm_bf16<64, AK, BK, EPI>), grid, dim3(256), 0, n->stream, g);
  }
  if (nsplit > 1)
    hipLaunchKernelGGL(k_gemm_splitk_reduce<EPI>, dim3((mn + 255) / 256), dim3(256), 0, n->stream, g, nsplit);
}

// forward of B rows from the bfloat16 input a[0] (already staged); y = out_scale * output
int run_forward(pdf_mlp* n, int B, float out_scale, float* y_out) {
  for (int l = 0; l < n->L; ++l) {
    GemmArgs g{};
    g.A = n->a[l];
    g.lda = n->sz[l];
    g.B = n->Wb[l];
    g.ldb = n->sz[l];
    g.Mr = B;
    g.Nc = n->sz[l + 1];
    g.K = n->sz[l];
    g.bias = n->b[l];
    g.ldc = n->sz[l + 1];
    if (l < n->L - 1) {
      g.C = n->z[l];
      g.Cb = n->a[l + 1];
      launch_gemm<true, true, EPI_BIAS_GELU>(n, g);
    } else {
      g.C = y_out ? y_out : n->z[l];
      g.out_scale = out_scale;
      launch_gemm<true, true, EPI_BIAS>(n, g);
    }
  }
  return mcheck(n, "forward");
}

int stage_input(pdf_mlp* n, const float* x, const int* idx, int nrows, float s_in, int B) {
  const size_t e = size_t(B) * n->sz[0];
  hipLaunchKernelGGL(k_input_bf16, dim3((e + 255) / 256), dim3(256), 0, n->stream, x, idx, nrows, s_in, B,
                     n->sz[0], n->a[0]);
  return mcheck(n, "input");
}

}  // namespace

extern "C" int pdf_mlp_create(int32_t n_layers, const int32_t* sizes, int32_t batch_max, void* stream,
                              pdf_mlp** out) {
  if (!sizes || !out || !stream || n_layers < 1 || n_layers > 16 || batch_max < 1)
    return mfail(nullptr, PDF_EINVAL, "pdf_mlp_create: bad argument");
  for (int l = 0; l <= n_layers; ++l)
    if (sizes[l] < 1 || sizes[l] > (1 << 20)) return mfail(nullptr, PDF_EINVAL, "pdf_mlp_create: bad layer width");
  pdf_mlp* n = new pdf_mlp();
  n->L = n_layers;
  n->bmax = batch_max;
  n->sz.assign(sizes, sizes + n_layers + 1);
  n->stream = (hipStream_t)stream;
  const int L = n->L;
  n->W.resize(L); n->b.resize(L); n->gW.resize(L); n->gb.resize(L);
  n->mW.resize(L); n->vW.resize(L); n->mb.resize(L); n->vb.resize(L); n->Wb.resize(L);
  n->a.resize(L); n->z.resize(L);
  int maxw = 0;
  int rc = PDF_OK;
  for (int l = 0; l < L && !rc; ++l) {
    const size_t nw = size_t(n->sz[l + 1]) * n->sz[l], nb = n->sz[l + 1];
    maxw = std::max(maxw, std::max(n->sz[l], n->sz[l + 1]));
    rc = rc ? rc : dalloc(n, &n->W[l], nw);
    rc = rc ? rc : dalloc(n, &n->gW[l], nw);
    rc = rc ? rc : dalloc(n, &n->mW[l], nw);
    rc = rc ? rc : dalloc(n, &n->vW[l], nw);
    rc = rc ? rc : dalloc(n, &n->Wb[l], nw);
    rc = rc ? rc : dalloc(n, &n->b[l], nb);
    rc = rc ? rc : dalloc(n, &n->gb[l], nb);
    rc = rc ? rc : dalloc(n, &n->mb[l], nb);
    rc = rc ? rc : dalloc(n, &n->vb[l], nb);
    rc = rc ? rc : dalloc(n, &n->a[l], size_t(batch_max) * n->sz[l]);
    rc = rc ? rc : dalloc(n, &n->z[l], size_t(batch_max) * n->sz[l + 1]);
  }
  for (int q = 0; q < 2; ++q) {
    rc = rc ? rc : dalloc(n, &n->dz[q], size_t(batch_max) * maxw);
    rc = rc ? rc : dalloc(n, &n->dzb[q], size_t(batch_max) * maxw);
  }
  rc = rc ? rc : dalloc(n, &n->part, kMlpSplitFloats);
  rc = rc ? rc : dalloc(n, &n->rowsum, batch_max);
  rc = rc ? rc : dalloc(n, &n->loss, 1);
  if (rc) {
    pdf_mlp_destroy(n);
    return rc;
  }
  for (int l = 0; l < L; ++l) {
    const size_t nw = size_t(n->sz[l + 1]) * n->sz[l], nb = n->sz[l + 1];
    for (float* p : {n->W[l], n->mW[l], n->vW[l], n->gW[l]}) (void)hipMemsetAsync(p, 0, sizeof(float) * nw, n->stream);
    for (float* p : {n->b[l], n->mb[l], n->vb[l], n->gb[l]}) (void)hipMemsetAsync(p, 0, sizeof(float) * nb, n->stream);
    (void)hipMemsetAsync(n->Wb[l], 0, sizeof(u16) * nw, n->stream);
  }
  if (hipStreamSynchronize(n->stream) != hipSuccess) {
    pdf_mlp_destroy(n);
    return mfail(nullptr, PDF_EHIP, "pdf_mlp_create: stream failed");
  }
  *out = n;
  return PDF_OK;
}

extern "C" void pdf_mlp_destroy(pdf_mlp* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  for (void* p : n->owned) (void)hipFree(p);
  delete n;
}

extern "C" int pdf_mlp_set_layer(pdf_mlp* n, int32_t l, const float* W_host, const float* b_host) {
  if (!n || l < 0 || l >= n->L || !W_host || !b_host) return mfail(n, PDF_EINVAL, "pdf_mlp_set_layer: bad argument");
  const size_t nw = size_t(n->sz[l + 1]) * n->sz[l], nb = n->sz[l + 1];
  if (hipMemcpyAsync(n->W[l], W_host, sizeof(float) * nw, hipMemcpyHostToDevice, n->stream) != hipSuccess ||
      hipMemcpyAsync(n->b[l], b_host, sizeof(float) * nb, hipMemcpyHostToDevice, n->stream) != hipSuccess)
    return mfail(n, PDF_EHIP, "pdf_mlp_set_layer: copy failed");
  for (float* p : {n->mW[l], n->vW[l]}) (void)hipMemsetAsync(p, 0, sizeof(float) * nw, n->stream);
  for (float* p : {n->mb[l], n->vb[l]}) (void)hipMemsetAsync(p, 0, sizeof(float) * nb, n->stream);
  hipLaunchKernelGGL(k_to_bf16, dim3((nw + 255) / 256), dim3(256), 0, n->stream, n->W[l], n->Wb[l], nw);
  n->t = 0;
  if (int rc = mcheck(n, "pdf_mlp_set_layer")) return rc;
  if (hipStreamSynchronize(n->stream) != hipSuccess) return mfail(n, PDF_EHIP, "pdf_mlp_set_layer: sync failed");
  return PDF_OK;
}

extern "C" int pdf_mlp_get_layer(pdf_mlp* n, int32_t l, int32_t what, float* W_host, float* b_host) {
  if (!n || l < 0 || l >= n->L || !W_host || !b_host || what < 0 || what > 1)
    return mfail(n, PDF_EINVAL, "pdf_mlp_get_layer: bad argument");
  const size_t nw = size_t(n->sz[l + 1]) * n->sz[l], nb = n->sz[l + 1];
  const float* sw = what == 0 ? n->W[l] : n->gW[l];
  const float* sb = what == 0 ? n->b[l] : n->gb[l];
  if (hipMemcpyAsync(W_host, sw, sizeof(float) * nw, hipMemcpyDeviceToHost, n->stream) != hipSuccess ||
      hipMemcpyAsync(b_host, sb, sizeof(float) * nb, hipMemcpyDeviceToHost, n->stream) != hipSuccess ||
      hipStreamSynchronize(n->stream) != hipSuccess)
    return mfail(n, PDF_EHIP, "pdf_mlp_get_layer: copy failed");
  return PDF_OK;
}

extern "C" int pdf_mlp_forward(pdf_mlp* n, const float* x_dev, float s_in, float s_out, int32_t B, float* y_dev) {
  if (!n || !x_dev || !y_dev || B < 1 || B > n->bmax) return mfail(n, PDF_EINVAL, "pdf_mlp_forward: bad argument");
  if (int rc = stage_input(n, x_dev, nullptr, B, s_in, B)) return rc;
  return run_forward(n, B, s_out, y_dev);
}

extern "C" int pdf_mlp_train_step(pdf_mlp* n, const float* x_dev, const float* t_dev, int32_t n_rows,
                                  const int32_t* idx_dev, float s_in, int32_t B, double lr, double* loss_dev) {
  if (!n || !x_dev || !t_dev || B < 1 || B > n->bmax || !(lr > 0) || n_rows < 1 || (!idx_dev && n_rows < B))
    return mfail(n, PDF_EINVAL, "pdf_mlp_train_step: bad argument");
  const int L = n->L, nout = n->sz[L];
  if (int rc = stage_input(n, x_dev, idx_dev, n_rows, s_in, B)) return rc;
  if (int rc = run_forward(n, B, 1.0f, nullptr)) return rc;
  int cur = 0;
  hipLaunchKernelGGL(k_mse, dim3(B), dim3(256), 0, n->stream, n->z[L - 1], t_dev, idx_dev, n_rows, B, nout,
                     n->dz[cur], n->dzb[cur], n->rowsum);
  hipLaunchKernelGGL(k_mse_total, dim3(1), dim3(64), 0, n->stream, n->rowsum, B, nout, loss_dev ? loss_dev : n->loss);
  for (int l = L - 1; l >= 0; --l) {
    const int no = n->sz[l + 1], ni = n->sz[l];
    {  // gW[o][i] = sum_b dz[b][o] a[b][i]: rows o, columns i, reduction over the batch
      GemmArgs g{};
      g.A = n->dzb[cur];
      g.lda = no;
      g.B = n->a[l];
      g.ldb = ni;
      g.Mr = no;
      g.Nc = ni;
      g.K = B;
      g.C = n->gW[l];
      g.ldc = ni;
      launch_gemm<false, false, EPI_STORE>(n, g);
    }
    hipLaunchKernelGGL(k_colsum, dim3((no + 15) / 16), dim3(256), 0, n->stream, n->dz[cur], B, no, n->gb[l]);
    if (l > 0) {  // dz_prev[b][i] = gelu'(z_prev) * sum_o dz[b][o] W[o][i]
      GemmArgs g{};
      g.A = n->dzb[cur];
      g.lda = no;
      g.B = n->Wb[l];
      g.ldb = ni;
      g.Mr = B;
      g.Nc = ni;
      g.K = no;
      g.C = n->dz[1 - cur];
      g.Cb = n->dzb[1 - cur];
      g.ldc = ni;
      g.zprev = n->z[l - 1];
      launch_gemm<true, false, EPI_GELU_GRAD>(n, g);
      cur = 1 - cur;
    }
  }
  n->t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float lr1 = float(lr / (1.0 - std::pow(0.9, n->t)));
  const float ic2 = float(1.0 / (1.0 - std::pow(0.999, n->t)));
  for (int l = 0; l < L; ++l) {
    const size_t nw = size_t(n->sz[l + 1]) * n->sz[l], nb = n->sz[l + 1];
    hipLaunchKernelGGL(k_adam, dim3((nw + 255) / 256), dim3(256), 0, n->stream, n->W[l], n->gW[l], n->mW[l],
                       n->vW[l], n->Wb[l], nw, lr1, b1, b2, ic2, eps);
    hipLaunchKernelGGL(k_adam, dim3((nb + 255) / 256), dim3(256), 0, n->stream, n->b[l], n->gb[l], n->mb[l],
                       n->vb[l], (u16*)nullptr, nb, lr1, b1, b2, ic2, eps);
  }
  return mcheck(n, "pdf_mlp_train_step");
}

hipStream_t pdf_mlp_stream(const pdf_mlp* n) { return n->stream; }

extern "C" int pdf_mlp_widths(const pdf_mlp* n, int32_t* n_in, int32_t* n_out, int32_t* batch_max) {
  if (!n) return PDF_EINVAL;
  if (n_in) *n_in = n->sz[0];
  if (n_out) *n_out = n->sz[n->L];
  if (batch_max) *batch_max = n->bmax;
  return PDF_OK;
}
