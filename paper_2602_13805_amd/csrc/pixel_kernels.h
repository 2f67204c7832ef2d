// Per-pixel and per-instance kernels: the reduction over incidences that
// yields the CIE contrast and the state loss, the receiver GEMMs, the
// regularisers with their gradient, the CCO image, and small reductions.
#pragma once

#include <type_traits>

#include "cplx.h"

namespace pdfk {

// Deterministic sum over a block (fixed tree).  red: >= blockDim.x/64 doubles of LDS.
__device__ __forceinline__ double block_sum(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;  // valid in thread 0
}

__device__ __forceinline__ double block_max(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_down(x, o, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s = fmax(s, red[i]);
  }
  return s;
}

template <typename T>
struct ReduceArgs {
  const cx<T>* J;       // [B][Ni][N]
  const cx<T>* E;       // [B][Ni][N]
  const cx<T>* gs;      // [Ns][N]
  const cx<T>* gsT;     // [N][Ns] (the same operator, receiver-contiguous)
  const float* gsA;     // FP32 MFMA path: [N][ceil(Ns/16)][64] A operands in lane order (see below)
  const cx<T>* Rfix;    // [B][N] fixed contrast, or null (least squares)
  cx<T>* R;             // [B][N] out (least squares only)
  T* den;               // [B][N] out
  cx<T>* chi;           // [B][N] out
  double* lsp;          // [B][ntiles] out: partial sum_p |R E_p - beta J_p|^2
  cx<T>* Dpart;         // [B][ntiles][Ni][Ns] out: partial G_S J over the tile
  double* wsum;         // null, or [B][N][4] out: wgt (Re num, Im num, den, sum |J|^2) per pixel
  double wgt;
  int Ni, Ns, N, ntiles;
  T beta;
};

// Tile of pixels x all incidences of one instance (grid: ntiles x B).
//   num = sum_p J conj(E), den = sum_p |E|^2 (FP64 accumulation)
//   R = beta num / den (Eq. 6 solved per pixel), chi = R / (beta (1 - R)) (Eq. 7)
//   sum_p |R E - beta J|^2 = |R|^2 den - 2 beta Re(R conj(num)) + beta^2 sum |J|^2
//   Dpart[p][q] = sum_{n in tile} G_S[q][n] J_p[n]   (split-K part of Eq. 16)
template <typename T>
__global__ __launch_bounds__(256) void k_pixel_reduce(ReduceArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TILE = blockDim.x;
  cx<T>* Jt = reinterpret_cast<cx<T>*>(smem_raw);  // [Ni][TILE]
  double* red = reinterpret_cast<double*>(Jt + size_t(a.Ni) * TILE);
  const int tile = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int n = tile * TILE + tid;
  const bool valid = n < a.N;
  double nr = 0, ni = 0, dd = 0, jj = 0;
  for (int p = 0; p < a.Ni; ++p) {
    cx<T> J{T(0), T(0)}, E{T(0), T(0)};
    if (valid) {
      const size_t idx = (size_t(b) * a.Ni + p) * a.N + n;
      J = a.J[idx];
      E = a.E[idx];
    }
    nr += double(J.x) * E.x + double(J.y) * E.y;
    ni += double(J.y) * E.x - double(J.x) * E.y;
    dd += double(E.x) * E.x + double(E.y) * E.y;
    jj += double(J.x) * J.x + double(J.y) * J.y;
    Jt[size_t(p) * TILE + tid] = J;
  }
  double lpix = 0.0;
  if (valid) {
    const double beta = a.beta;
    double rr, ri;
    if (a.Rfix) {
      const cx<T> r = a.Rfix[size_t(b) * a.N + n];
      rr = r.x;
      ri = r.y;
    } else {
      rr = beta * nr / dd;
      ri = beta * ni / dd;
      a.R[size_t(b) * a.N + n] = cx<T>{T(rr), T(ri)};
    }
    // sum_p |R E_p - beta J_p|^2
    lpix = (rr * rr + ri * ri) * dd - 2.0 * beta * (rr * nr + ri * ni) + beta * beta * jj;
    a.den[size_t(b) * a.N + n] = T(dd);
    if (a.wsum) {
      double* ws = a.wsum + (size_t(b) * a.N + n) * 4;
      ws[0] = a.wgt * nr;
      ws[1] = a.wgt * ni;
      ws[2] = a.wgt * dd;
      ws[3] = a.wgt * jj;
    }
    // chi = R / (beta (1 - R))
    const double xr = 1.0 - rr, xi = -ri;
    const double q = beta * (xr * xr + xi * xi);
    a.chi[size_t(b) * a.N + n] = cx<T>{T((rr * xr + ri * xi) / q), T((ri * xr - rr * xi) / q)};
  }
  const double s = block_sum(lpix, red);
  if (tid == 0) a.lsp[size_t(b) * a.ntiles + tile] = s;
  __syncthreads();
  const int tile0 = tile * TILE;
  const int kmax = min(TILE, a.N - tile0);
  for (int o = tid; o < a.Ni * a.Ns; o += TILE) {
    const int p = o / a.Ns, q = o % a.Ns;
    const cx<T>* g = a.gs + size_t(q) * a.N + tile0;
    const cx<T>* jt = Jt + size_t(p) * TILE;
    cx<T> acc{T(0), T(0)};
    for (int k = 0; k < kmax; ++k) acc = acc + g[k] * jt[k];
    a.Dpart[((size_t(b) * a.ntiles + tile) * a.Ni + p) * a.Ns + q] = acc;
  }
}


typedef float floatx16 __attribute__((ext_vector_type(16)));

// FP32 version of k_pixel_reduce with the split-K receiver GEMM on MFMA.
// Block: 256 threads over a tile of 256 pixels, taken as two sub-tiles of
// 128 so that the staging LDS stays near 34 KB and four blocks share a CU.
// Per sub-tile:
//  1. the reduction over incidences: thread (pixel, half) loads the
//     incidences p = half, half + 2, ... of its pixel in batches of PB
//     (loads issued before use), accumulates num / den / sum |J|^2 in FP64
//     and stages J in LDS; the two halves are added in fixed order;
//  2. the complex GEMM D[p][q] += sum_k G_S[q][k] J_p[k] over the sub-tile
//     as a real GEMM C = A B with A the 2x2-block real form of G_S (rows
//     2q+c: c = 0 real, 1 imaginary part of D) and B the (Re, Im) rows of J:
//       A[2q][2k] = Re G, A[2q][2k+1] = -Im G, A[2q+1][2k] = Im G, A[2q+1][2k+1] = Re G.
//     One v_mfma_f32_32x32x2f32 consumes one complex pixel for a 32 x 32
//     output tile (16 receivers x 32 incidences); each wave takes a quarter
//     of the sub-tile.
// The four waves' partial tiles are summed through LDS in fixed order.
// NRT = ceil(Ns / 16) row tiles, NCT = ceil(Ni / 32) column tiles.
constexpr int kReduceTile = 256, kReduceSub = 128;

template <int NCT>
constexpr size_t reduce_mfma_lds() {
  return sizeof(float) * 2 * kReduceSub * (32 * NCT + 1) + sizeof(double) * 4 * kReduceSub + 16 * sizeof(double);
}

// PB: incidences per load batch (a tuning choice: the accumulation order does
// not depend on it, so neither do the results).
template <int NRT, int NCT, int PB>
__device__ __forceinline__ void pixel_reduce_mfma_body(const ReduceArgs<float>& a, int tile, int b,
                                                       unsigned char* smem_raw) {
  constexpr int SUB = kReduceSub, NSUB = kReduceTile / kReduceSub;
  constexpr int LDJ = 32 * NCT + 1;  // padded row of the staged currents (floats)
  float* Jr = reinterpret_cast<float*>(smem_raw);         // [SUB][LDJ]
  float* Ji = Jr + SUB * LDJ;                               // [SUB][LDJ]
  double* part = reinterpret_cast<double*>(Ji + SUB * LDJ);  // [4][SUB] sums of the second half
  double* red = part + 4 * SUB;
  const int tid = threadIdx.x;
  const int Ni = a.Ni, Ns = a.Ns, N = a.N;
  const int px = tid & (SUB - 1), half = tid / SUB;
  const int lane = tid & 63, w = tid >> 6;
  const int m = lane & 31, cp = lane >> 5;    // A row within the tile / k component (0 Re J, 1 Im J)
  const float* Jsrc = cp ? Ji : Jr;
  const double beta = a.beta;
  floatx16 acc[NRT][NCT];
#pragma unroll
  for (int h = 0; h < NRT; ++h)
#pragma unroll
    for (int t = 0; t < NCT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[h][t][r] = 0.f;
  double lpix = 0.0;

  for (int sub = 0; sub < NSUB; ++sub) {
    const int sub0 = tile * kReduceTile + sub * SUB;
    if (sub0 >= N) break;  // block-uniform
    const int n = sub0 + px;
    const bool valid = n < N;
    // 1. reduction over this thread's incidences
    double nr = 0, ni = 0, dd = 0, jj = 0;
    const int nc = min(n, N - 1);
    // the instance's blocks (workgroup-uniform) and 32-bit byte offsets (8 Ni N <= 8 x 64 x 256^2)
    const char* Jb = reinterpret_cast<const char*>(a.J + size_t(b) * Ni * N);
    const char* Eb = reinterpret_cast<const char*>(a.E + size_t(b) * Ni * N);
    auto ld = [&](const char* base, int p) {
      return *reinterpret_cast<const cx<float>*>(base + 8u * unsigned(p * N + nc));
    };
    // Loaded values are used unconditionally (in a sub-tile past the end, a
    // pixel beyond it is masked by a multiplication): a load whose value feeds
    // only one arm of a select is moved under a branch by the compiler and
    // waited for on its own.
    const float vm = valid ? 1.f : 0.f;
    int p0 = half;
    // the sub-tile's incidences; MASK: the sub-tile reaches past the end (a block-uniform choice)
    auto incidences = [&](auto mask_c) {
      constexpr bool MASK = decltype(mask_c)::value;
      // each sum is a chain of FP64 fused multiply-adds, in the same order for every load batch
      auto accumulate = [&](int p, cx<float> J, cx<float> E) {
        if constexpr (MASK) {
          J = cx<float>{vm * J.x, vm * J.y};
          E = cx<float>{vm * E.x, vm * E.y};
        }
        const double jx = J.x, jy = J.y, ex = E.x, ey = E.y;
        nr = fma(jy, ey, fma(jx, ex, nr));
        ni = fma(-jx, ey, fma(jy, ex, ni));
        dd = fma(ey, ey, fma(ex, ex, dd));
        jj = fma(jy, jy, fma(jx, jx, jj));
        Jr[px * LDJ + p] = J.x;
        Ji[px * LDJ + p] = J.y;
      };
      for (; p0 + 2 * (PB - 1) < Ni; p0 += 2 * PB) {  // whole batches: loads issued before use
        cx<float> Jv[PB], Ev[PB];
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          Jv[u] = ld(Jb, p0 + 2 * u);
          Ev[u] = ld(Eb, p0 + 2 * u);
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) accumulate(p0 + 2 * u, Jv[u], Ev[u]);
      }
      for (; p0 < Ni; p0 += 2) accumulate(p0, ld(Jb, p0), ld(Eb, p0));
    };
    if (sub0 + SUB <= N)
      incidences(std::false_type{});
    else
      incidences(std::true_type{});
    for (; p0 < 32 * NCT; p0 += 2) {  // zero incidences pad the MFMA tile
      Jr[px * LDJ + p0] = 0.f;
      Ji[px * LDJ + p0] = 0.f;
    }
    if (half == 1) {
      part[px] = nr;
      part[SUB + px] = ni;
      part[2 * SUB + px] = dd;
      part[3 * SUB + px] = jj;
    }
    __syncthreads();  // staged J and the second half's sums are complete
    if (half == 0 && valid) {
      nr += part[px];
      ni += part[SUB + px];
      dd += part[2 * SUB + px];
      jj += part[3 * SUB + px];
      double rr, ri;
      if (a.Rfix) {
        const cx<float> r = a.Rfix[size_t(b) * N + n];
        rr = r.x;
        ri = r.y;
      } else {
        rr = beta * nr / dd;
        ri = beta * ni / dd;
        a.R[size_t(b) * N + n] = cx<float>{float(rr), float(ri)};
      }
      lpix += (rr * rr + ri * ri) * dd - 2.0 * beta * (rr * nr + ri * ni) + beta * beta * jj;
      a.den[size_t(b) * N + n] = float(dd);
      if (a.wsum) {
        double* ws = a.wsum + (size_t(b) * N + n) * 4;
        ws[0] = a.wgt * nr;
        ws[1] = a.wgt * ni;
        ws[2] = a.wgt * dd;
        ws[3] = a.wgt * jj;
      }
      const double xr = 1.0 - rr, xi = -ri;
      const double q = beta * (xr * xr + xi * xi);
      a.chi[size_t(b) * N + n] = cx<float>{float((rr * xr + ri * xi) / q), float((ri * xr - rr * xi) / q)};
    }
    // 2. receiver GEMM over this sub-tile.  The A operands come precomputed
    // per (pixel, row tile) in lane order: lane l = m + 32 cp holds
    // sgn * (Re or Im) G_S[q][n] for q = 16 h + m / 2, or 0 for a padding
    // receiver, so each is one coalesced load at a constant stride; the next
    // chunk's loads are issued before this chunk's MFMAs
    const int kmax = min(SUB, N - sub0);
    const int k0 = w * (SUB / 4), k1 = min(k0 + SUB / 4, kmax);
    constexpr int KC = 4;
    if (k1 - k0 == SUB / 4) {  // a whole quarter (wave-uniform): no clamping or masking, constant offsets
      const float* Ab = a.gsA + (size_t(sub0) + k0) * NRT * 64 + lane;
      const float* Bb = Jsrc + k0 * LDJ + m;
#pragma unroll
      for (int kk = 0; kk < SUB / 4; ++kk) {
        float av[NRT], bv[NCT];
#pragma unroll
        for (int h = 0; h < NRT; ++h) av[h] = Ab[(kk * NRT + h) * 64];
#pragma unroll
        for (int t = 0; t < NCT; ++t) bv[t] = Bb[kk * LDJ + 32 * t];
#pragma unroll
        for (int h = 0; h < NRT; ++h)
#pragma unroll
          for (int t = 0; t < NCT; ++t)
            acc[h][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[h], bv[t], acc[h][t], 0, 0, 0);
      }
    } else if (k0 < k1) {  // wave-uniform
      const float* Ab = a.gsA + size_t(sub0) * NRT * 64 + lane;
      // pixels past the range (clamped loads) are masked by a zero operand
      auto load_a = [&](float (&av)[KC][NRT], int kb) {
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
          const int k = kb + kk;
          const float in = k < k1 ? 1.f : 0.f;
          const int kc = k < k1 ? k : k0;
#pragma unroll
          for (int h = 0; h < NRT; ++h) av[kk][h] = in * Ab[(size_t(kc) * NRT + h) * 64];
        }
      };
      float av[KC][NRT];
      load_a(av, k0);
      for (int kb = k0; kb < k1; kb += KC) {
        float an[KC][NRT], bv[KC][NCT];
        load_a(an, kb + KC);  // past the end: clamped, masked, unused
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
          const int k = kb + kk;
#pragma unroll
          for (int t = 0; t < NCT; ++t) bv[kk][t] = Jsrc[(k < k1 ? k : k0) * LDJ + 32 * t + m];
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
#pragma unroll
          for (int h = 0; h < NRT; ++h)
#pragma unroll
            for (int t = 0; t < NCT; ++t)
              acc[h][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[kk][h], bv[kk][t], acc[h][t], 0, 0, 0);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
#pragma unroll
          for (int h = 0; h < NRT; ++h) av[kk][h] = an[kk][h];
      }
    }
    __syncthreads();  // the staging buffers are rewritten by the next sub-tile
  }
  const double s = block_sum(lpix, red);
  if (tid == 0) a.lsp[size_t(b) * a.ntiles + tile] = s;

  // sum the four waves' partial tiles (reusing the staging LDS) and store
  float* W = Jr;  // [4][16][64] floats per output tile
  cx<float>* Dout = a.Dpart + (size_t(b) * a.ntiles + tile) * Ni * Ns;
#pragma unroll
  for (int h = 0; h < NRT; ++h)
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) W[(w * 16 + r) * 64 + lane] = acc[h][t][r];
      __syncthreads();
      for (int e = tid; e < 1024; e += 256) {
        const float v = W[e] + W[1024 + e] + W[2048 + e] + W[3072 + e];
        const int r = e >> 6, l = e & 63;
        const int i = (r & 3) + 8 * (r >> 2) + 4 * (l >> 5);   // row of the 32 x 32 tile
        const int q = 16 * h + (i >> 1), p = 32 * t + (l & 31);
        if (q < Ns && p < Ni) reinterpret_cast<float*>(Dout + p * Ns + q)[i & 1] = v;
      }
    }
}

template <int NRT, int NCT, int PB>
__global__ __launch_bounds__(256, (NRT * NCT <= 2 && PB <= 4 ? 4 : 2)) void k_pixel_reduce_mfma(ReduceArgs<float> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  pixel_reduce_mfma_body<NRT, NCT, PB>(a, blockIdx.x, blockIdx.y, smem_raw);
}

// One launch over several argument sets of one shape class (the same tile
// count ntiles); set g's workgroup l is tile l % ntiles of instance l / ntiles.
template <int NRT, int NCT, int PB>
__global__ __launch_bounds__(256, (NRT * NCT <= 2 && PB <= 4 ? 4 : 2)) void k_pixel_reduce_mfma_group(
    const ReduceArgs<float>* __restrict__ a, const int* __restrict__ start, int n, int ntiles) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = group_of(start, n, blockIdx.x);
  const int l = blockIdx.x - start[g];
  pixel_reduce_mfma_body<NRT, NCT, PB>(a[g], l % ntiles, l / ntiles, smem_raw);
}

template <typename T>
struct RegArgs {
  int nfreq;            // > 1: L^Data = sum_f dn[f] / sdf[f] (per-frequency residual norms given)
  const double* dn;     // [nfreq] ||G_S,f J_f - E_sca,f||^2
  const double* sdf;    // [nfreq] ||E_sca,f||^2
  const cx<T>* chi;     // [B][N]
  const cx<T>* R;       // [B][N]
  const cx<T>* Dpart;   // [B][ntiles][Ni][Ns]
  const double* lsp;    // [B][ntiles]
  const cx<T>* esca;    // [B][Ni][Ns]
  const double* Ss;     // scalar
  const double* Sd;     // [B]
  cx<T>* d;             // [B][Ni][Ns] out: G_S J - E_sca
  cx<T>* gR;            // [B][N] out
  double* loss;         // [B][8] out, or null
  int* tstep;           // [B] incremented when non-null
  const int* frozen;    // [B] or null
  double* adam_c;       // [B][2] out with tstep: lr / (1 - b1^t), 1 / (1 - b2^t) at the new step t
  double lr, b1, b2;
  int M, Ni, Ns, ntiles;
  double beta, lam_bound, lam_tv, lam_bridge, tau_b, eps_tv, eps_abs;
  int r_stopgrad;
  // the loss on the CCO image: chi is chi_c, L^State gains the nlse sums lse
  // [B][nlse] (over ||E_inc||^2 like the rest), and gR receives dL/dchi_c of
  // the regularisers unconverted (graw)
  const double* lse;
  int nlse, graw;
};

template <typename T>
__device__ __forceinline__ T sigm(T x) { return T(1) / (T(1) + exp(-x)); }

// Regulariser terms anchored at pixel (i, j): value and the partial
// gradients with respect to chi(i,j), chi(i,j+1), chi(i+1,j) (Eqs. 17-19).
template <typename T>
struct RegTerm {
  double val_bound, val_tv, val_bridge;
  cx<T> g_self, g_right, g_down;  // weighted by the lambdas
};

template <typename T>
__device__ __forceinline__ RegTerm<T> reg_term(const cx<T>* c, int i, int j, int M, const RegArgs<T>& a) {
  RegTerm<T> r;
  const cx<T> z = c[i * M + j];
  const bool hr = j + 1 < M, hd = i + 1 < M;
  const cx<T> zr = hr ? c[i * M + j + 1] : z;
  const cx<T> zd = hd ? c[(i + 1) * M + j] : z;
  // bound
  const T neg = z.x < T(0) ? -z.x : T(0);
  r.val_bound = double(neg) * neg;
  cx<T> gs{T(-2 * a.lam_bound) * neg, T(0)};
  // total variation
  const cx<T> dx = zr - z, dy = zd - z;
  const T t = sqrt(norm2(dx) + norm2(dy) + T(a.eps_tv));
  r.val_tv = t;
  const T wt = T(a.lam_tv) / t;
  cx<T> gr = wt * dx, gd = wt * dy;
  gs = gs - wt * (dx + dy);
  // bridge, on the smoothed modulus a = sqrt(|chi|^2 + eps_abs)
  const T e = T(a.eps_abs), tb = T(a.tau_b);
  const T az = sqrt(norm2(z) + e), ar = sqrt(norm2(zr) + e), ad = sqrt(norm2(zd) + e);
  const T ax = hr ? ar - az : T(0), ay = hd ? ad - az : T(0);
  const T sg = sigm((az - tb) / tb);
  const T ex = exp(-ax * ax - ay * ay);
  r.val_bridge = double(sg) * ex;
  const T lb = T(a.lam_bridge);
  const T ga = lb * (sg * (T(1) - sg) / tb * ex + T(2) * sg * ex * (ax + ay));
  gs = gs + (ga / az) * z;
  if (hr) gr = gr + (lb * T(-2) * ax * sg * ex / ar) * zr;
  if (hd) gd = gd + (lb * T(-2) * ay * sg * ex / ad) * zd;
  r.g_self = gs;
  r.g_right = gr;
  r.g_down = gd;
  return r;
}

// Step counter and this step's Adam bias corrections of instance b (thread 0
// of one block), counted here so that the adjoint's Adam epilogue reads them
// instead of evaluating them in every thread.
template <typename T>
__device__ __forceinline__ void reg_count_step(const RegArgs<T>& a, int b) {
  if (a.tstep && !(a.frozen && a.frozen[b])) {
    const int t = a.tstep[b] + 1;
    a.tstep[b] = t;
    a.adam_c[2 * b] = a.lr / (1.0 - pow(a.b1, double(t)));
    a.adam_c[2 * b + 1] = 1.0 / (1.0 - pow(a.b2, double(t)));
  }
}

// Data residual d = G_S J - E_sca of output o of instance b from the split-K
// parts; returns |d|^2.
template <typename T>
__device__ __forceinline__ double reg_data(const RegArgs<T>& a, int b, int o, int NO) {
  double xr = 0.0, xi = 0.0;
  for (int t = 0; t < a.ntiles; ++t) {
    const cx<T> v = a.Dpart[(size_t(b) * a.ntiles + t) * NO + o];
    xr += v.x;
    xi += v.y;
  }
  const cx<T> e = a.esca[size_t(b) * NO + o];
  const double rr = xr - e.x, ri = xi - e.y;
  a.d[size_t(b) * NO + o] = cx<T>{T(rr), T(ri)};
  return rr * rr + ri * ri;
}

// g_R = conj(1 / (beta (1 - R)^2)) g_chi at pixel n from g_chi = g (g itself
// with graw, zero with R held fixed); tracks max |R| and non-finite gradients.
template <typename T>
__device__ __forceinline__ void reg_grad_out(const RegArgs<T>& a, int b, int n, const cx<T>& R, const cx<T>& g,
                                             double& rmax, bool& bad) {
  const int N = a.M * a.M;
  rmax = fmax(rmax, sqrt(double(norm2(R))));
  cx<T> gR{T(0), T(0)};
  if (a.graw) {
    gR = g;
  } else if (!a.r_stopgrad) {
    const cx<T> om{T(1) - R.x, -R.y};
    const cx<T> w = om * om;
    const T den = T(a.beta) * norm2(w);
    gR = cx<T>{(w.x * g.x - w.y * g.y) / den, (w.x * g.y + w.y * g.x) / den};
  }
  if (!(isfinite(gR.x) && isfinite(gR.y))) bad = true;
  a.gR[size_t(b) * N + n] = gR;
}

// The regularisers anchored at pixel n of the image c (Eqs. 17-19): adds their
// values to vb, vt, vr and writes g_R from their gradient g_chi at n (its own
// terms, then those anchored at its left and upper neighbours).
template <typename T>
__device__ __forceinline__ void reg_pixel(const RegArgs<T>& a, const cx<T>* c, int b, int n, double& vb, double& vt,
                                          double& vr, double& rmax, bool& bad) {
  const int M = a.M, N = M * M;
  const int i = n / M, j = n % M;
  RegTerm<T> t0 = reg_term<T>(c, i, j, M, a);
  vb += t0.val_bound;
  vt += t0.val_tv;
  vr += t0.val_bridge;
  cx<T> g = t0.g_self;
  if (j > 0) g = g + reg_term<T>(c, i, j - 1, M, a).g_right;
  if (i > 0) g = g + reg_term<T>(c, i - 1, j, M, a).g_down;
  reg_grad_out(a, b, n, a.R[size_t(b) * N + n], g, rmax, bad);
}

// The loss row of instance b from the block sums (thread 0); ls: the sum of
// the state-loss parts lsp and lse (before the division by ||E_inc||^2).
template <typename T>
__device__ __forceinline__ void reg_finish(const RegArgs<T>& a, int b, double ls, double Sd, double Sb, double St,
                                           double Sr, double Rm, double nb) {
  if (!a.loss) return;
  ls /= a.Ss[0];
  double ld = 0.0;
  if (a.nfreq > 1)
    for (int f = 0; f < a.nfreq; ++f) ld += a.dn[f] / a.sdf[f];
  else
    ld = Sd / a.Sd[b];
  const double tot = ls + ld + a.lam_bound * Sb + a.lam_tv * St + a.lam_bridge * Sr;
  double* L = a.loss + size_t(b) * 8;
  L[0] = ls;
  L[1] = ld;
  L[2] = Sb;
  L[3] = St;
  L[4] = Sr;
  L[5] = tot;
  L[6] = Rm;
  L[7] = (isfinite(tot) && nb == 0.0) ? 0.0 : 1.0;
}

// Pixels per thread of the one-workgroup regulariser: grids up to 96 x 96 in
// FP32 and 64 x 64 in FP64 at 1024 threads (larger ones take k_image_reg_part).
template <typename T>
constexpr int reg_pix_max() { return sizeof(T) == 4 ? 9 : 4; }

// One instance per block: data residual and L^Data from the split-K parts,
// L^State from its partial sums, the three regularisers on chi with their
// gradient g_chi, and g_R = conj(1 / (beta (1 - R)^2)) g_chi.  chi staged in
// LDS.  Each pixel's terms are evaluated once; the parts of their gradient that
// belong to the right and lower neighbours reach those through LDS, and each
// pixel adds them in the same order as evaluating the neighbours' terms again.
// LDS: 2 N complex values and 16 doubles; N <= reg_pix_max<T>() x blockDim.x.
template <typename T>
__device__ __forceinline__ void image_reg_body(const RegArgs<T>& a, int b, unsigned char* smem_raw) {
  constexpr int PMAX = reg_pix_max<T>();
  const int M = a.M, N = M * M;
  cx<T>* cs = reinterpret_cast<cx<T>*>(smem_raw);   // chi [M][M], then the g_down parts
  cx<T>* xs = cs + N;                                // the g_right parts
  double* red = reinterpret_cast<double*>(xs + N);
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) reg_count_step(a, b);
  for (int n = tid; n < N; n += nt) cs[n] = a.chi[size_t(b) * N + n];
  cx<T> Rv[PMAX], g[PMAX], gd[PMAX];
#pragma unroll
  for (int q = 0; q < PMAX; ++q) {
    const int n = tid + q * nt;
    Rv[q] = n < N ? a.R[size_t(b) * N + n] : cx<T>{T(0), T(0)};
  }
  double dsum = 0.0;
  const int NO = a.nfreq > 1 ? 0 : a.Ni * a.Ns;
  for (int o = tid; o < NO; o += nt) dsum += reg_data(a, b, o, NO);
  __syncthreads();
  double vb = 0, vt = 0, vr = 0, rmax = 0;
  bool bad = false;
#pragma unroll
  for (int q = 0; q < PMAX; ++q) {
    const int n = tid + q * nt;
    g[q] = gd[q] = cx<T>{T(0), T(0)};
    if (n < N) {
      const RegTerm<T> t = reg_term<T>(cs, n / M, n % M, M, a);
      vb += t.val_bound;
      vt += t.val_tv;
      vr += t.val_bridge;
      g[q] = t.g_self;
      gd[q] = t.g_down;
      xs[n] = t.g_right;
    }
  }
  __syncthreads();  // chi read, every g_right written
#pragma unroll
  for (int q = 0; q < PMAX; ++q) {
    const int n = tid + q * nt;
    if (n < N) {
      if (n % M > 0) g[q] = g[q] + xs[n - 1];
      cs[n] = gd[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PMAX; ++q) {
    const int n = tid + q * nt;
    if (n < N) {
      if (n >= M) g[q] = g[q] + cs[n - M];
      reg_grad_out(a, b, n, Rv[q], g[q], rmax, bad);
    }
  }
  const double Sd = block_sum(dsum, red);
  const double Sb = block_sum(vb, red);
  const double St = block_sum(vt, red);
  const double Sr = block_sum(vr, red);
  const double Rm = block_max(rmax, red);
  const double nb = block_sum(bad ? 1.0 : 0.0, red);
  if (tid == 0 && a.loss) {
    double ls = 0.0;
    for (int t = 0; t < a.ntiles; ++t) ls += a.lsp[size_t(b) * a.ntiles + t];
    for (int t = 0; t < a.nlse; ++t) ls += a.lse[size_t(b) * a.nlse + t];
    reg_finish(a, b, ls, Sd, Sb, St, Sr, Rm, nb);
  }
}

// Images beyond one workgroup's LDS: chi read from global memory, 256 pixels
// (and data outputs) per workgroup of a grid (nblk, B); each workgroup's sums
// (|d|^2, bound, TV, bridge, max |R|, non-finite count) go to part[B][nblk][6]
// and k_image_reg_fin adds them in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_image_reg_part(RegArgs<T> a, double* __restrict__ part) {
  __shared__ double red[16];
  const int M = a.M, N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * 256 + threadIdx.x;
  const int NO = a.nfreq > 1 ? 0 : a.Ni * a.Ns;
  double dsum = 0.0;
  for (int o = n; o < NO; o += gridDim.x * 256) dsum += reg_data(a, b, o, NO);
  double vb = 0, vt = 0, vr = 0, rmax = 0;
  bool bad = false;
  if (n < N) reg_pixel(a, a.chi + size_t(b) * N, b, n, vb, vt, vr, rmax, bad);
  const double v[6] = {block_sum(dsum, red), block_sum(vb, red), block_sum(vt, red), block_sum(vr, red),
                       block_max(rmax, red), block_sum(bad ? 1.0 : 0.0, red)};
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) part[(size_t(b) * gridDim.x + blockIdx.x) * 6 + k] = v[k];
}

// The loss rows and step counters from k_image_reg_part's sums and the
// state-loss parts, each added by 256 threads (every 256th part) and a fixed
// tree.  Grid B, 256 threads.
template <typename T>
__global__ __launch_bounds__(256) void k_image_reg_fin(RegArgs<T> a, const double* __restrict__ part, int nblk) {
  __shared__ double red[16];
  const int b = blockIdx.x, tid = threadIdx.x;
  double s[6] = {0, 0, 0, 0, 0, 0}, ls = 0.0;
  for (int k = tid; k < nblk; k += 256) {
    const double* p = part + (size_t(b) * nblk + k) * 6;
    for (int q = 0; q < 6; ++q) s[q] = q == 4 ? fmax(s[q], p[q]) : s[q] + p[q];
  }
  for (int t = tid; t < a.ntiles; t += 256) ls += a.lsp[size_t(b) * a.ntiles + t];
  for (int t = tid; t < a.nlse; t += 256) ls += a.lse[size_t(b) * a.nlse + t];
  double S[6];
  for (int q = 0; q < 6; ++q) S[q] = q == 4 ? block_max(s[q], red) : block_sum(s[q], red);
  const double L = block_sum(ls, red);
  if (tid == 0) {
    reg_count_step(a, b);
    reg_finish(a, b, L, S[0], S[1], S[2], S[3], S[4], S[5]);
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_image_reg(RegArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  image_reg_body<T>(a, blockIdx.x, smem_raw);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_image_reg_group(const RegArgs<T>* __restrict__ a,
                                                          const int* __restrict__ start, int n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = group_of(start, n, blockIdx.x);
  image_reg_body<T>(a[g], blockIdx.x - start[g], smem_raw);
}

// h[b][p][n] = s * sum_q conj(G_S[q][n]) x[b][p][q]   (G_S^H applied to Ns-vectors)
// Grid: (ceil(N / 256), B), block 256; the G_S column of a pixel sits in registers.
template <typename T, int NSMAX>
__global__ __launch_bounds__(256) void k_adj_gemm(const cx<T>* __restrict__ gs, const cx<T>* __restrict__ x,
                                                  cx<T>* __restrict__ h, int Ni, int Ns, int N) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* xs = reinterpret_cast<cx<T>*>(smem_raw);  // [Ni][Ns]
  const int b = blockIdx.y, tid = threadIdx.x;
  for (int o = tid; o < Ni * Ns; o += blockDim.x) xs[o] = x[size_t(b) * Ni * Ns + o];
  __syncthreads();
  const int n = blockIdx.x * blockDim.x + tid;
  if (n >= N) return;
  cx<T> g[NSMAX];
#pragma unroll
  for (int q = 0; q < NSMAX; ++q) g[q] = q < Ns ? gs[size_t(q) * N + n] : cx<T>{T(0), T(0)};
  for (int p = 0; p < Ni; ++p) {
    cx<T> acc{T(0), T(0)};
#pragma unroll
    for (int q = 0; q < NSMAX; ++q) {
      if (q < Ns) acc = acc + cmul_conj_a(g[q], xs[p * Ns + q]);
    }
    h[(size_t(b) * Ni + p) * N + n] = acc;
  }
}

// FP32 version of k_adj_gemm on MFMA: for one instance, the real-expanded
// GEMM D = A B with rows i = 2p + c (c = 0 real, 1 imaginary part of h_p),
// columns the pixels and one receiver q per K step of two:
//   A[2p][2q] = Re x, A[2p][2q+1] = Im x, A[2p+1][2q] = Im x, A[2p+1][2q+1] = -Re x,
//   B[2q][n] = Re G_S[q][n], B[2q+1][n] = Im G_S[q][n],
// so that D[2p][n] + i D[2p+1][n] = sum_q conj(G_S[q][n]) x[p][q].
// Block: 4 waves x CT column tiles of 32 pixels; x^T is staged in LDS
// (incidence-contiguous, conflict-free reads); each lane of a finished tile
// holds (Re, Im) of h_p at one pixel, so stores are 256-byte rows.
// Requires N % 32 == 0.  NRT = ceil(Ni / 16) row tiles; CT column tiles of 32
// pixels per wave (a tuning choice: every output is the same chain of MFMAs
// over the receivers whatever CT is, so the results do not depend on it).
struct AdjGemmArgs {
  const cx<float>* gs;  // [Ns][N]
  const cx<float>* x;   // [B][Ni][Ns]
  cx<float>* h;         // [B][Ni][N] out
  int Ni, Ns, N;
};

template <int NRT, int CT>
__device__ __forceinline__ void adj_gemm_mfma_body(const AdjGemmArgs& args, int bx, int b, unsigned char* smem_raw) {
  constexpr int KC = 8, LDX = 16 * NRT;
  const cx<float>* __restrict__ gs = args.gs;
  const cx<float>* __restrict__ x = args.x;
  cx<float>* __restrict__ h = args.h;
  const int Ni = args.Ni, Ns = args.Ns, N = args.N;
  cx<float>* xs = reinterpret_cast<cx<float>*>(smem_raw);  // [Ns][LDX]: xs[q][p] = x[p][q]
  const int tid = threadIdx.x;
  for (int o = tid; o < Ns * LDX; o += blockDim.x) {
    const int q = o / LDX, p = o % LDX;
    xs[o] = p < Ni ? x[(size_t(b) * Ni + p) * Ns + q] : cx<float>{0.f, 0.f};
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int m = lane & 31, cp = lane >> 5;
  const int c = m & 1;
  const int n0 = (bx * 4 + w) * 32 * CT;
  const float* Gf = reinterpret_cast<const float*>(gs);
  // the wave's CT column tiles one after another: a tile's stores drain while
  // the next tile's loads and MFMAs run, and only one tile's accumulators
  // are live (each output sums over the receivers in the same order)
  for (int t = 0; t < CT; ++t) {
    const int nt0 = n0 + 32 * t;
    if (nt0 >= N) break;  // wave-uniform; no barrier follows
    floatx16 acc[NRT];
#pragma unroll
    for (int r = 0; r < NRT; ++r)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[r][e] = 0.f;
    for (int qb = 0; qb < Ns; qb += KC) {
      float av[KC][NRT], bv[KC];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int q = qb + kk;
        const bool in = q < Ns;
        // unconditional loads from clamped (in-bounds) addresses, then a select
        // (a zero A operand masks receivers past Ns)
        const int qc = min(q, Ns - 1);
        bv[kk] = Gf[(size_t(qc) * N + nt0 + m) * 2 + cp];
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
          const cx<float> d = xs[qc * LDX + 16 * r + (m >> 1)];
          av[kk][r] = (in ? 1.f : 0.f) * (c == 0 ? (cp == 0 ? d.x : d.y) : (cp == 0 ? d.y : -d.x));
        }
      }
#pragma unroll
      for (int kk = 0; kk < KC; ++kk)
#pragma unroll
        for (int r = 0; r < NRT; ++r)
          acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[kk][r], bv[kk], acc[r], 0, 0, 0);
    }
    // lane (l % 32 = pixel, l / 32) holds rows i = (e % 4) + 8 (e / 4) + 4 (l / 32): pairs (e, e + 1)
    // with e even are (Re, Im) of incidence p = 16 r + i / 2
#pragma unroll
    for (int r = 0; r < NRT; ++r)
#pragma unroll
      for (int e = 0; e < 16; e += 2) {
        const int i = (e & 3) + 8 * (e >> 2) + 4 * cp;
        const int p = 16 * r + (i >> 1);
        if (p < Ni) h[(size_t(b) * Ni + p) * N + nt0 + m] = cx<float>{acc[r][e], acc[r][e + 1]};
      }
  }
}

template <int NRT, int CT>
__global__ __launch_bounds__(256) void k_adj_gemm_mfma(const cx<float>* __restrict__ gs,
                                                       const cx<float>* __restrict__ x, cx<float>* __restrict__ h,
                                                       int Ni, int Ns, int N) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  adj_gemm_mfma_body<NRT, CT>(AdjGemmArgs{gs, x, h, Ni, Ns, N}, blockIdx.x, blockIdx.y, smem_raw);
}

// Grouped: set g's workgroup l is pixel block l % nbx of instance l / nbx.
template <int NRT, int CT>
__global__ __launch_bounds__(256) void k_adj_gemm_mfma_group(const AdjGemmArgs* __restrict__ a,
                                                             const int* __restrict__ start, int n, int nbx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = group_of(start, n, blockIdx.x);
  const int l = blockIdx.x - start[g];
  adj_gemm_mfma_body<NRT, CT>(a[g], l % nbx, l / nbx, smem_raw);
}

// s[b] = sum |x[b][*]|^2 over len entries (grid: B blocks).
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const cx<T>* x, size_t len, double* s) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < len; i += blockDim.x) {
    const cx<T> v = x[size_t(b) * len + i];
    acc += double(v.x) * v.x + double(v.y) * v.y;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) s[b] = t;
}

// Count-normalised (2r+1)^2 box mean of an M x M array in LDS.
template <typename T>
__device__ __forceinline__ T box_mean(const T* x, int i, int j, int M, int r) {
  T s = T(0);
  int cnt = 0;
  for (int di = -r; di <= r; ++di) {
    const int ii = i + di;
    if (ii < 0 || ii >= M) continue;
    for (int dj = -r; dj <= r; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= M) continue;
      s += x[ii * M + jj];
      ++cnt;
    }
  }
  return s / T(cnt);
}

template <typename T>
struct CcoArgs {
  const cx<T>* chi;        // [B][N]
  cx<T>* out;              // [B][N] CCO image, or null
  const cx<T>* eps_true;   // [B][N] or null
  double* err;             // [B] or null
  int M, r;
  double gf_eps, tau, eta_max, delta;
};

// CCO (Sec. 2.4, Eqs. 10-11): chi_cco = (1 + eta) G(chi|chi) + eta chi with the
// self-guided filter G on Re and Im separately and
// eta = eta_max sigmoid((|chi| - tau) / delta); optional relative error of
// 1 + chi_cco against the true permittivity.  One instance per block of
// min(N, 1024) threads, each with at most kCcoPix pixels (N <= 9216).  LDS
// holds Re chi, Im chi and the filter coefficients A, b of one part at a
// time: the real part is filtered first and kept in registers.
constexpr int kCcoPix = 9;

template <typename T>
__device__ __forceinline__ void gf_coeffs(const T* p, T* A, T* bb, int M, int r, T ge, int tid, int nt) {
  const int N = M * M;
  for (int n = tid; n < N; n += nt) {
    const int i = n / M, j = n % M;
    T s = 0, s2 = 0;
    int cnt = 0;
    for (int di = -r; di <= r; ++di) {
      const int ii = i + di;
      if (ii < 0 || ii >= M) continue;
      for (int dj = -r; dj <= r; ++dj) {
        const int jj = j + dj;
        if (jj < 0 || jj >= M) continue;
        const T v = p[ii * M + jj];
        s += v;
        s2 += v * v;
        ++cnt;
      }
    }
    const T mu = s / T(cnt);
    const T var = s2 / T(cnt) - mu * mu;
    const T a = var / (var + ge);
    A[n] = a;
    bb[n] = (T(1) - a) * mu;
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_cco(CcoArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int M = a.M, N = M * M;
  T* pr = reinterpret_cast<T*>(smem_raw);  // Re chi, Im chi, A and b of the part being filtered
  T* pi = pr + N;
  T* A = pi + N;
  T* bb = A + N;
  double* red = reinterpret_cast<double*>(bb + N);
  const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  for (int n = tid; n < N; n += nt) {
    const cx<T> z = a.chi[size_t(b) * N + n];
    pr[n] = z.x;
    pi[n] = z.y;
  }
  __syncthreads();
  const T ge = T(a.gf_eps);
  gf_coeffs(pr, A, bb, M, a.r, ge, tid, nt);
  __syncthreads();
  T gr[kCcoPix];
#pragma unroll
  for (int k = 0; k < kCcoPix; ++k) {
    const int n = tid + k * nt;
    gr[k] = T(0);
    if (n < N) gr[k] = box_mean(A, n / M, n % M, M, a.r) * pr[n] + box_mean(bb, n / M, n % M, M, a.r);
  }
  __syncthreads();  // A and b are rewritten for the imaginary part
  gf_coeffs(pi, A, bb, M, a.r, ge, tid, nt);
  __syncthreads();
  double enum_ = 0, eden = 0;
#pragma unroll
  for (int k = 0; k < kCcoPix; ++k) {
    const int n = tid + k * nt;
    if (n >= N) continue;
    const int i = n / M, j = n % M;
    const T gi = box_mean(A, i, j, M, a.r) * pi[n] + box_mean(bb, i, j, M, a.r);
    const T mag = sqrt(pr[n] * pr[n] + pi[n] * pi[n]);
    const T eta = T(a.eta_max) / (T(1) + exp(-(mag - T(a.tau)) / T(a.delta)));
    const cx<T> o{(T(1) + eta) * gr[k] + eta * pr[n], (T(1) + eta) * gi + eta * pi[n]};
    if (a.out) a.out[size_t(b) * N + n] = o;
    if (a.eps_true) {
      const cx<T> e = a.eps_true[size_t(b) * N + n];
      const double dr = double(T(1) + o.x) - e.x, di = double(o.y) - e.y;
      enum_ += dr * dr + di * di;
      eden += double(e.x) * e.x + double(e.y) * e.y;
    }
  }
  if (a.err) {
    const double s1 = block_sum(enum_, red);
    const double s2 = block_sum(eden, red);
    if (tid == 0) a.err[b] = sqrt(s1 / s2);
  }
}

}  // namespace pdfk
