// The per-incidence steps of the loss for grids whose padded half tile does
// not fit one CU's LDS (FP32 above 96 x 96, FP64 above 64 x 64): the same
// operations as conv_kernels.h (basis synthesis, the 2x-padded FFT
// convolution with the domain operator, the CIE bracket, the adjoint with the
// basis analysis and Adam), split into passes that exchange through a global
// array S of the M stored rows of each padded spectrum, [BP][M][P]:
//   rows:    J rows (synthesised from alpha, or given), zero-padded to P,
//            length-P FFT along x                          -> S
//   columns: each column's M stored entries, zero-padded, length-P FFT along
//            y, times the spectrum of G_D (conjugated for the adjoint),
//            inverse, cropped to M                          -> S
//   rows:    inverse length-P FFT along x, cropped to M, epilogue.
// Each pass is a batch of 1-D transforms on LDS tiles (fft_lds.h): RB rows or
// CB columns per workgroup.  The workgroups of an instance-incidence pair sit
// on one XCD in every pass (xcd_remap), so S passes between them through that
// XCD's L2 where it fits.
#pragma once

#include "conv_kernels.h"
#include "cplx.h"
#include "fft_lds.h"
#include "pixel_kernels.h"

namespace pdfk {

template <typename T, int M_>
struct BigCfg {
  static constexpr int M = M_, P = 2 * M, N = M * M;
  static constexpr bool TRI = M % 3 == 0;
  static constexpr int NT = 256;                                  // threads of the row passes
  static constexpr int EPT_P = TRI ? 12 : (P >= 512 ? 16 : 8);     // length-P row transforms
  static constexpr int RB = NT * EPT_P / P;                       // rows per workgroup
  static constexpr int EPT_M = TRI ? 12 : (M >= 256 ? 16 : 8);     // length-M row transforms
  static constexpr int CB = 16;                                   // columns per workgroup
  static constexpr int EPT_C = TRI ? 12 : 16;
  static constexpr int NTC = CB * P / EPT_C;                      // threads of the column pass
  static_assert(M % RB == 0 && P % CB == 0 && NTC % 64 == 0 && NTC <= 1024, "big-grid tiling");
  static constexpr int RBLK = M / RB;                             // row workgroups per pair
  static constexpr int CBLK = P / CB;                             // column workgroups per pair
  using Rows = Vecs<P, RB, true>;
  using Cols = Vecs<CB, CB, false>;
  static constexpr size_t ROW_LDS = sizeof(cx<T>) * (size_t(RB) * (P + 1) + P);
  static constexpr size_t COL_LDS = sizeof(cx<T>) * (size_t(P) * (CB + 1) + P);
};

// exp(+2 pi i k m / M) from the P-point table tw[k] = exp(-2 pi i k / P)
template <typename T>
__device__ __forceinline__ cx<T> tw_inv_m(const cx<T>* tw, int km, int P) {
  int e = (-2 * km) % P;
  e += e < 0 ? P : 0;
  return tw[e];
}

// Rows pass of the forward convolution for RB rows of pair bp: J rows (from the
// K x K coefficients: U[i][kx] = sum_ky alpha[ky][kx] exp(2 pi i ky i / M), then
// a zero-filled inverse length-M FFT along x; or the given currents), written
// to a.J when synthesised, then the zero-padded length-P FFT along x into S.
template <typename T, int M, bool FROM_ALPHA>
__global__ __launch_bounds__(256) void k_big_rows_fwd(FwdArgs<T> a, cx<T>* __restrict__ S) {
  using C = BigCfg<T, M>;
  constexpr int P = C::P, RB = C::RB, LD = P + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + RB * LD;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int bp = blk / C::RBLK, i0 = (blk % C::RBLK) * RB;
  const int tid = threadIdx.x;
  for (int k = tid; k < P; k += C::NT) tw[k] = a.tw[k];
  if constexpr (FROM_ALPHA) {
    for (int e = tid; e < RB * LD; e += C::NT) buf[e] = cx<T>{T(0), T(0)};
    __syncthreads();
    const int K = a.K, KK = K * K, kmin = -(K / 2);
    const cx<T>* al = a.in + size_t(bp) * KK;
    for (int e = tid; e < RB * K; e += C::NT) {
      const int r = e / K, kxi = e % K, i = i0 + r;
      cx<T> u{T(0), T(0)};
      for (int kyi = 0; kyi < K; ++kyi) u = u + al[kyi * K + kxi] * tw_inv_m(tw, (kmin + kyi) * i, P);
      buf[r * LD + wrap_mode(kmin + kxi, M)] = u;
    }
    __syncthreads();
    Fft<T, M, C::EPT_M, C::NT, typename C::Rows, 2>{buf, tw, typename C::Rows{}}.template run<+1>();
    for (int e = tid; e < RB * M; e += C::NT) {
      const int r = e / M, j = e % M;
      a.J[size_t(bp) * C::N + size_t(i0 + r) * M + j] = buf[r * LD + j];
    }
  } else {
    for (int e = tid; e < RB * M; e += C::NT) {
      const int r = e / M, j = e % M;
      buf[r * LD + j] = a.in[size_t(bp) * C::N + size_t(i0 + r) * M + j];
    }
    __syncthreads();
  }
  Fft<T, P, C::EPT_P, C::NT, typename C::Rows, 1>{buf, tw, typename C::Rows{}}.template run<-1, M, P>();
  for (int e = tid; e < RB * P; e += C::NT) {
    const int r = e / P, k = e % P;
    S[(size_t(bp) * M + i0 + r) * P + k] = buf[r * LD + k];
  }
}

// Columns pass for CB columns of pair bp: the M stored entries of each column
// of S, zero-padded, length-P FFT along y, times ghat (its conjugate for the
// adjoint), inverse, cropped to M, back into S.
template <typename T, int M>
__global__ __launch_bounds__((BigCfg<T, M>::NTC)) void k_big_cols(const cx<T>* __restrict__ ghat,
                                                                const cx<T>* __restrict__ twg, cx<T>* __restrict__ S,
                                                                int adjoint) {
  using C = BigCfg<T, M>;
  constexpr int P = C::P, CB = C::CB, LD = CB + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + P * LD;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int bp = blk / C::CBLK, c0 = (blk % C::CBLK) * CB;
  const int tid = threadIdx.x;
  for (int k = tid; k < P; k += C::NTC) tw[k] = twg[k];
  for (int e = tid; e < M * CB; e += C::NTC) {
    const int i = e / CB, c = e % CB;
    buf[i * LD + c] = S[(size_t(bp) * M + i) * P + c0 + c];
  }
  __syncthreads();
  using F = Fft<T, P, C::EPT_C, C::NTC, typename C::Cols, 1>;
  F{buf, tw, typename C::Cols{}}.template run<-1, M, P>();
  for (int e = tid; e < P * CB; e += C::NTC) {
    const int k = e / CB, c = e % CB;
    cx<T> w = ghat[size_t(k) * P + c0 + c];
    if (adjoint) w.y = -w.y;
    buf[k * LD + c] = buf[k * LD + c] * w;
  }
  __syncthreads();
  F{buf, tw, typename C::Cols{}}.template run<+1, P, M>();
  for (int e = tid; e < M * CB; e += C::NTC) {
    const int i = e / CB, c = e % CB;
    S[(size_t(bp) * M + i) * P + c0 + c] = buf[i * LD + c];
  }
}

// Last rows pass of the forward convolution: inverse length-P FFT along x,
// cropped to M, and E = E_inc + G_D J + beta J (Sec. 2.2, Eq. 6).
template <typename T, int M, bool FROM_ALPHA>
__global__ __launch_bounds__(256) void k_big_rows_inv(FwdArgs<T> a, const cx<T>* __restrict__ S) {
  using C = BigCfg<T, M>;
  constexpr int P = C::P, RB = C::RB, LD = P + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + RB * LD;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int bp = blk / C::RBLK, i0 = (blk % C::RBLK) * RB, p = bp % a.Ni;
  const int tid = threadIdx.x;
  for (int k = tid; k < P; k += C::NT) tw[k] = a.tw[k];
  for (int e = tid; e < RB * P; e += C::NT) {
    const int r = e / P, k = e % P;
    buf[r * LD + k] = S[(size_t(bp) * M + i0 + r) * P + k];
  }
  __syncthreads();
  Fft<T, P, C::EPT_P, C::NT, typename C::Rows, 1>{buf, tw, typename C::Rows{}}.template run<+1, P, M>();
  const cx<T>* Jsrc = FROM_ALPHA ? a.J : a.in;
  for (int e = tid; e < RB * M; e += C::NT) {
    const int r = e / M, j = e % M;
    const size_t n = size_t(i0 + r) * M + j;
    const cx<T> jv = Jsrc[size_t(bp) * C::N + n];
    const cx<T> ei = a.einc ? a.einc[size_t(p) * C::N + n] : cx<T>{T(0), T(0)};
    a.E[size_t(bp) * C::N + n] = buf[r * LD + j] + a.beta * jv + ei;
  }
}

// Adjoint, first rows pass: the per-pixel part of the chain rule (as in
// adj_conv_body), g_E into the tile and g_J into GJ, then the zero-padded
// length-P FFT of g_E along x into S.
template <typename T, int M>
__global__ __launch_bounds__(256) void k_big_adj_rows(AdjArgs<T> a, cx<T>* __restrict__ S, cx<T>* __restrict__ GJ) {
  using C = BigCfg<T, M>;
  constexpr int P = C::P, RB = C::RB, LD = P + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + RB * LD;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int bp = blk / C::RBLK, i0 = (blk % C::RBLK) * RB;
  const int b = bp / a.Ni, p = bp % a.Ni;
  const int tid = threadIdx.x;
  const size_t off = size_t(bp) * C::N, eoff = size_t(a.e_shared ? p : bp) * C::N, boff = size_t(b) * C::N;
  const T ws = T(2) / T(a.Ss[0]);
  const T wd = T(2 * a.hsign) / T(a.Sd[b]);
  const T beta = a.beta;
  for (int k = tid; k < P; k += C::NT) tw[k] = a.tw[k];
  for (int e = tid; e < RB * M; e += C::NT) {
    const int r = e / M, j = e % M;
    const size_t n = size_t(i0 + r) * M + j;
    const cx<T> J = a.J ? a.J[off + n] : cx<T>{T(0), T(0)};
    const cx<T> E = a.E[eoff + n], R = a.R[boff + n];
    const cx<T> s = R * E - beta * J;
    const cx<T> gs = ws * s;
    cx<T> gE = cmul_conj_a(R, gs);
    cx<T> gJ = (-beta) * gs + wd * a.h[off + n];
    if (a.gR) {
      const cx<T> g = a.gR[boff + n];
      const T inv = a.gr_w / a.den[boff + n];
      const T re = g.x * R.x + g.y * R.y;  // Re(conj(g) R)
      gE = gE + inv * (beta * cmul_conj_a(g, J) - (T(2) * re) * E);
      gJ = gJ + (beta * inv) * (g * E);
    }
    gJ = gJ + beta * gE;
    buf[r * LD + j] = gE;
    GJ[off + n] = gJ;
  }
  __syncthreads();
  Fft<T, P, C::EPT_P, C::NT, typename C::Rows, 1>{buf, tw, typename C::Rows{}}.template run<-1, M, P>();
  for (int e = tid; e < RB * P; e += C::NT) {
    const int r = e / P, k = e % P;
    S[(size_t(bp) * M + i0 + r) * P + k] = buf[r * LD + k];
  }
}

// Adjoint, last rows pass: inverse length-P FFT along x cropped to M (G_D^H
// g_E), plus g_J, then the forward length-M FFT along x of the sum; the K kept
// columns of each row go to the first K entries of the row's S (V[i][kx]).
// GJ == nullptr: the input rows are taken from x as they are (no convolution
// result, no g_J): the analysis of given pixel arrays.
template <typename T, int M, bool CONV>
__global__ __launch_bounds__(256) void k_big_adj_rows_inv(const cx<T>* __restrict__ twg, cx<T>* __restrict__ S,
                                                          const cx<T>* __restrict__ GJ, int K) {
  using C = BigCfg<T, M>;
  constexpr int P = C::P, RB = C::RB, LD = P + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + RB * LD;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int bp = blk / C::RBLK, i0 = (blk % C::RBLK) * RB;
  const int tid = threadIdx.x;
  for (int k = tid; k < P; k += C::NT) tw[k] = twg[k];
  if constexpr (CONV) {
    for (int e = tid; e < RB * P; e += C::NT) {
      const int r = e / P, k = e % P;
      buf[r * LD + k] = S[(size_t(bp) * M + i0 + r) * P + k];
    }
    __syncthreads();
    Fft<T, P, C::EPT_P, C::NT, typename C::Rows, 1>{buf, tw, typename C::Rows{}}.template run<+1, P, M>();
    for (int e = tid; e < RB * M; e += C::NT) {
      const int r = e / M, j = e % M;
      buf[r * LD + j] = buf[r * LD + j] + GJ[size_t(bp) * C::N + size_t(i0 + r) * M + j];
    }
  } else {
    for (int e = tid; e < RB * M; e += C::NT) {
      const int r = e / M, j = e % M;
      buf[r * LD + j] = GJ[size_t(bp) * C::N + size_t(i0 + r) * M + j];
    }
  }
  __syncthreads();
  Fft<T, M, C::EPT_M, C::NT, typename C::Rows, 2>{buf, tw, typename C::Rows{}}.template run<-1>();
  const int kmin = -(K / 2);
  for (int e = tid; e < RB * K; e += C::NT) {
    const int r = e / K, kxi = e % K;
    S[(size_t(bp) * M + i0 + r) * P + kxi] = buf[r * LD + wrap_mode(kmin + kxi, M)];
  }
}

// Adjoint, last pass, gridDim.y workgroups per pair (each a share of the kept
// rows): the forward DFT along y of the K kept columns, restricted to the K
// kept rows, g_alpha[ky][kx] = sum_i V[i][kx] exp(-2 pi i ky i / M) (g_alpha =
// B^H g_J), then the gradient output and the Adam update exactly as in the
// LDS-resident adjoint.  scale multiplies the result (1 for the gradient;
// 1 / M^2 for the analysis F_T).
template <typename T, int M>
__global__ __launch_bounds__(256) void k_big_adj_final(AdjArgs<T> a, const cx<T>* __restrict__ S, T scale) {
  using C = BigCfg<T, M>;
  constexpr int P = C::P;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  const int bp = xcd_remap(blockIdx.x, gridDim.x), b = bp / a.Ni;
  const int tid = threadIdx.x;
  for (int k = tid; k < P; k += blockDim.x) tw[k] = a.tw[k];
  __syncthreads();
  const int K = a.K, kmin = -(K / 2);
  const bool upd = a.alpha && !(a.frozen && a.frozen[b]);
  T lr1 = T(0), ic2 = T(0);
  if (upd) {
    lr1 = T(a.adam_c[2 * b]);
    ic2 = T(a.adam_c[2 * b + 1]);
  }
  const int rows = (K + gridDim.y - 1) / gridDim.y, r0 = blockIdx.y * rows, r1 = min(K, r0 + rows);
  for (int e = r0 * K + tid; e < r1 * K; e += blockDim.x) {
    const int ky = kmin + e / K, kxi = e % K;
    cx<T> g{T(0), T(0)};
    for (int i = 0; i < M; ++i) {
      int x = (2 * ky * i) % P;
      x += x < 0 ? P : 0;
      g = g + S[(size_t(bp) * M + i) * P + kxi] * tw[x];
    }
    g = scale * g;
    const size_t idx = size_t(bp) * K * K + e;
    if (a.galpha) a.galpha[idx] = g;
    if (upd) {
      const T b1 = T(a.b1), b2 = T(a.b2);
      T m0 = b1 * a.m[2 * idx] + (T(1) - b1) * g.x;
      T m1 = b1 * a.m[2 * idx + 1] + (T(1) - b1) * g.y;
      T v0 = b2 * a.v[2 * idx] + (T(1) - b2) * g.x * g.x;
      T v1 = b2 * a.v[2 * idx + 1] + (T(1) - b2) * g.y * g.y;
      a.m[2 * idx] = m0;
      a.m[2 * idx + 1] = m1;
      a.v[2 * idx] = v0;
      a.v[2 * idx + 1] = v1;
      const T eps = T(a.eps);
      cx<T> al = a.alpha[idx];
      al.x -= lr1 * m0 / (sqrt(v0 * ic2) + eps);
      al.y -= lr1 * m1 / (sqrt(v1 * ic2) + eps);
      a.alpha[idx] = al;
    }
  }
}

// ---- the CCO image for grids beyond one workgroup's LDS (Sec. 2.4, Eqs. 10-11)

// Self-guided filter coefficients of Re chi and Im chi per pixel (box of
// radius r, count-normalised at the edges): A = var / (var + eps), b = (1 - A) mu.
// w: [B][4][N] (A_re, b_re, A_im, b_im).  Grid (ceil(N / 256), B).
template <typename T>
__global__ __launch_bounds__(256) void k_cco_big_coef(const cx<T>* __restrict__ chi, T* __restrict__ w, int M, int r,
                                                      double gf_eps) {
  const int N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int i = n / M, j = n % M;
  const cx<T>* c = chi + size_t(b) * N;
  T sr = 0, sr2 = 0, si = 0, si2 = 0;
  int cnt = 0;
  for (int di = -r; di <= r; ++di) {
    const int ii = i + di;
    if (ii < 0 || ii >= M) continue;
    for (int dj = -r; dj <= r; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= M) continue;
      const cx<T> v = c[ii * M + jj];
      sr += v.x;
      sr2 += v.x * v.x;
      si += v.y;
      si2 += v.y * v.y;
      ++cnt;
    }
  }
  const T ge = T(gf_eps);
  T* wb = w + size_t(b) * 4 * N;
  const T mr = sr / T(cnt), vr = sr2 / T(cnt) - mr * mr, ar = vr / (vr + ge);
  const T mi = si / T(cnt), vi = si2 / T(cnt) - mi * mi, ai = vi / (vi + ge);
  wb[n] = ar;
  wb[N + n] = (T(1) - ar) * mr;
  wb[2 * N + n] = ai;
  wb[3 * N + n] = (T(1) - ai) * mi;
}

// chi_cco = (1 + eta) G + eta chi, G = mean(A) p + mean(b) per part, and the
// per-workgroup sums of the image error.  part: [B][gridDim.x][2] doubles.
template <typename T>
__global__ __launch_bounds__(256) void k_cco_big_apply(const cx<T>* __restrict__ chi, const T* __restrict__ w,
                                                       CcoArgs<T> a, double* __restrict__ part) {
  __shared__ double red[16];
  const int M = a.M, N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double en = 0.0, ed = 0.0;
  if (n < N) {
    const int i = n / M, j = n % M;
    const T* wb = w + size_t(b) * 4 * N;
    const cx<T> z = chi[size_t(b) * N + n];
    const T gr = box_mean(wb, i, j, M, a.r) * z.x + box_mean(wb + N, i, j, M, a.r);
    const T gi = box_mean(wb + 2 * N, i, j, M, a.r) * z.y + box_mean(wb + 3 * N, i, j, M, a.r);
    const T mag = sqrt(z.x * z.x + z.y * z.y);
    const T eta = T(a.eta_max) / (T(1) + exp(-(mag - T(a.tau)) / T(a.delta)));
    const cx<T> o{(T(1) + eta) * gr + eta * z.x, (T(1) + eta) * gi + eta * z.y};
    if (a.out) a.out[size_t(b) * N + n] = o;
    if (a.eps_true) {
      const cx<T> e = a.eps_true[size_t(b) * N + n];
      const double dr = double(T(1) + o.x) - e.x, di = double(o.y) - e.y;
      en = dr * dr + di * di;
      ed = double(e.x) * e.x + double(e.y) * e.y;
    }
  }
  const double s1 = block_sum(en, red);
  const double s2 = block_sum(ed, red);
  if (threadIdx.x == 0) {
    part[(size_t(b) * gridDim.x + blockIdx.x) * 2] = s1;
    part[(size_t(b) * gridDim.x + blockIdx.x) * 2 + 1] = s2;
  }
}

// err[b] = sqrt(sum of the parts in order).  Grid B, one thread.
__global__ void k_cco_big_err(const double* __restrict__ part, int nblk, double* __restrict__ err) {
  const int b = blockIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < nblk; ++k) {
    s1 += part[(size_t(b) * nblk + k) * 2];
    s2 += part[(size_t(b) * nblk + k) * 2 + 1];
  }
  err[b] = sqrt(s1 / s2);
}

}  // namespace pdfk
