// The loss evaluated on the CCO image (an option of the solver; the paper
// applies the contrast-compensated operator of Sec. 2.4, Eqs. 10-11, to the
// final image only).  With it every chi-dependent term of the loss (Sec. 3.2,
// Eqs. 13-19) sees chi_c = CCO(chi): the regularisers are evaluated on chi_c
// and the state residual takes R_c = beta chi_c / (1 + beta chi_c) (Eq. 7).
//
// Because R is the per-pixel least-squares optimum of the state residual,
//   L_State(R_c) = L_State(R) + sum_n den_n |R_c,n - R_n|^2 / ||E_inc||^2,
// (den = sum_p |E_p|^2), so the per-pixel sums the incidence reduction already
// formed are enough; its gradient in R_c is 2 den (R_c - R) / ||E_inc||^2.
// The gradient g_c with respect to chi_c (regularisers plus this state term
// through dR_c/dchi_c = beta / (1 + beta chi_c)^2) is taken back through the
// CCO to chi, then to R as in the plain path; the adjoint convolution kernel
// forms the state residual with R_c and the chain through R with R.
//
// The CCO's self-guided filter G(p) = mean(A) p + mean(b) acts on Re chi and
// Im chi separately (mu = mean(p), var = mean(p^2) - mu^2, A = var / (var +
// eps), b = (1 - A) mu; box means of radius r normalised by the in-grid count)
// and eta = eta_max sigmoid((|chi| - tau) / delta).  Its vector-Jacobian
// product takes these steps backwards; mean_t is the transpose of the box
// mean (each pixel collects x / cnt from the windows that contain it).
//
// Five stencil passes over the instances' images, each a grid of
// (ceil(N / 256), B) workgroups through a workspace [B][kCclArrays][N] of
// real images (the passes need their neighbours' values of the pass before):
//   coef  (mu, A, 1 - A, b per part)       apply (mean(A), chi_c, R_c, state sums)
//   adj1  (g_c, the sources of the two transposed means of the filter's last step)
//   adj2  (g_var, g_mu)                    adj3  (g_chi, g_R)
#pragma once

#include "cplx.h"
#include "pixel_kernels.h"

namespace pdfk {

// real images per instance in the workspace, two parts (Re, Im) each
enum CclArray { kCclMu = 0, kCclA = 2, kCclOA = 4, kCclB = 6, kCclBA = 8, kCclT1 = 10, kCclT2 = 12, kCclT3 = 14,
                kCclT4 = 16, kCclArrays = 18 };

template <typename T>
struct CcoLossArgs {
  const cx<T>* chi;   // [B][N] chi from the least-squares R
  const cx<T>* R;     // [B][N]
  const T* den;       // [B][N] sum_p |E_p|^2
  const double* Ss;   // ||E_inc||^2
  T* ws;              // [B][kCclArrays][N]
  cx<T>* chic;        // [B][N] chi_c
  cx<T>* Rc;          // [B][N] R_c
  double* part;       // [B][gridDim.x] sums of den |R_c - R|^2 per workgroup
  cx<T>* g;           // [B][N] in: dL/dchi_c of the regularisers; out: g_R
  double* loss;       // [B][8] or null: the non-finite flag of a bad gradient
  int M, r, r_stopgrad;
  double beta, gf_eps, tau, eta_max, delta;
};

// sum over the window of (i, j) of x[pixel] / cnt(pixel): the transpose of box_mean
template <typename T>
__device__ __forceinline__ T box_mean_t(const T* x, int i, int j, int M, int r) {
  T s = T(0);
  for (int di = -r; di <= r; ++di) {
    const int ii = i + di;
    if (ii < 0 || ii >= M) continue;
    const int ci = min(ii + r, M - 1) - max(ii - r, 0) + 1;
    for (int dj = -r; dj <= r; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= M) continue;
      const int cj = min(jj + r, M - 1) - max(jj - r, 0) + 1;
      s += x[ii * M + jj] / T(ci * cj);
    }
  }
  return s;
}

template <typename T>
__device__ __forceinline__ T ccl_eta(const CcoLossArgs<T>& a, T mag) {
  return T(a.eta_max) / (T(1) + exp(-(mag - T(a.tau)) / T(a.delta)));
}

// mu, A, 1 - A = eps / (var + eps) (formed directly: 1 - A would cancel where
// var >> eps) and b = (1 - A) mu of both parts
template <typename T>
__global__ __launch_bounds__(256) void k_ccl_coef(CcoLossArgs<T> a) {
  const int M = a.M, N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int i = n / M, j = n % M, r = a.r;
  const cx<T>* c = a.chi + size_t(b) * N;
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
  const T ge = T(a.gf_eps);
  T* w = a.ws + size_t(b) * kCclArrays * N;
  const T s[2] = {sr, si}, s2[2] = {sr2, si2};
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const T mu = s[ch] / T(cnt), var = s2[ch] / T(cnt) - mu * mu;
    const T oa = ge / (var + ge);
    w[(kCclMu + ch) * N + n] = mu;
    w[(kCclA + ch) * N + n] = var / (var + ge);
    w[(kCclOA + ch) * N + n] = oa;
    w[(kCclB + ch) * N + n] = oa * mu;
  }
}

// chi_c = (1 + eta) G + eta chi, R_c, mean(A) (kept for the adjoint) and the
// per-workgroup sums of den |R_c - R|^2
template <typename T>
__global__ __launch_bounds__(256) void k_ccl_apply(CcoLossArgs<T> a) {
  __shared__ double red[16];
  const int M = a.M, N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double ex = 0.0;
  if (n < N) {
    const int i = n / M, j = n % M;
    T* w = a.ws + size_t(b) * kCclArrays * N;
    const size_t o = size_t(b) * N + n;
    const cx<T> z = a.chi[o];
    const T bar = box_mean(w + kCclA * N, i, j, M, a.r), bai = box_mean(w + (kCclA + 1) * N, i, j, M, a.r);
    const T gr = bar * z.x + box_mean(w + kCclB * N, i, j, M, a.r);
    const T gi = bai * z.y + box_mean(w + (kCclB + 1) * N, i, j, M, a.r);
    w[kCclBA * N + n] = bar;
    w[(kCclBA + 1) * N + n] = bai;
    const T eta = ccl_eta(a, sqrt(z.x * z.x + z.y * z.y));
    const cx<T> c{(T(1) + eta) * gr + eta * z.x, (T(1) + eta) * gi + eta * z.y};
    a.chic[o] = c;
    // R_c = beta chi_c / (1 + beta chi_c)
    const T be = T(a.beta);
    const cx<T> bc{be * c.x, be * c.y};
    const cx<T> q{T(1) + bc.x, bc.y};
    const T qq = q.x * q.x + q.y * q.y;
    const cx<T> rc{(bc.x * q.x + bc.y * q.y) / qq, (bc.y * q.x - bc.x * q.y) / qq};
    a.Rc[o] = rc;
    const cx<T> R = a.R[o];
    const double dr = double(rc.x) - R.x, di = double(rc.y) - R.y;
    ex = double(a.den[o]) * (dr * dr + di * di);
  }
  const double s = block_sum(ex, red);
  if (threadIdx.x == 0) a.part[size_t(b) * gridDim.x + blockIdx.x] = s;
}

// g_c = dL/dchi_c: the regularisers' part (in g) plus the state term
// conj(beta / (1 + beta chi_c)^2) 2 den (R_c - R) / ||E_inc||^2, kept in g; the
// filter's output gradient u = (1 + eta) g_c per part, with u p and u for the
// transposed means of mean(A) p and mean(b)
template <typename T>
__global__ __launch_bounds__(256) void k_ccl_adj1(CcoLossArgs<T> a) {
  const int M = a.M, N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  T* w = a.ws + size_t(b) * kCclArrays * N;
  const size_t o = size_t(b) * N + n;
  const cx<T> z = a.chi[o], c = a.chic[o], rc = a.Rc[o], R = a.R[o];
  const T s = T(2.0 / a.Ss[0]) * a.den[o];
  const cx<T> gs{s * (rc.x - R.x), s * (rc.y - R.y)};
  // conj(beta / q^2), q = 1 + beta chi_c
  const T be = T(a.beta);
  const cx<T> q{T(1) + be * c.x, be * c.y};
  const cx<T> q2{q.x * q.x - q.y * q.y, T(2) * q.x * q.y};
  const T qq = q2.x * q2.x + q2.y * q2.y;
  const cx<T> f{be * q2.x / qq, be * q2.y / qq};  // conj(beta / q2) = beta q2 / |q2|^2
  cx<T> g = a.g[o];
  g = g + cx<T>{f.x * gs.x - f.y * gs.y, f.x * gs.y + f.y * gs.x};
  a.g[o] = g;
  const T eta = ccl_eta(a, sqrt(z.x * z.x + z.y * z.y));
  const T ur = (T(1) + eta) * g.x, ui = (T(1) + eta) * g.y;
  w[kCclT1 * N + n] = ur * z.x;
  w[(kCclT1 + 1) * N + n] = ui * z.y;
  w[kCclT2 * N + n] = ur;
  w[(kCclT2 + 1) * N + n] = ui;
}

// g_b = mean_t(u), g_A = mean_t(u p) - mu g_b, g_var = g_A (1 - A)^2 / eps,
// g_mu = (1 - A) g_b - 2 mu g_var, per part
template <typename T>
__global__ __launch_bounds__(256) void k_ccl_adj2(CcoLossArgs<T> a) {
  const int M = a.M, N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int i = n / M, j = n % M;
  T* w = a.ws + size_t(b) * kCclArrays * N;
  const T ge = T(a.gf_eps);
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const T gb = box_mean_t(w + (kCclT2 + ch) * N, i, j, M, a.r);
    const T mu = w[(kCclMu + ch) * N + n], oa = w[(kCclOA + ch) * N + n];
    const T gA = box_mean_t(w + (kCclT1 + ch) * N, i, j, M, a.r) - mu * gb;
    const T gvar = gA * (oa * oa / ge);
    w[(kCclT3 + ch) * N + n] = gvar;
    w[(kCclT4 + ch) * N + n] = oa * gb - T(2) * mu * gvar;
  }
}

// g_p = mean(A) u + 2 p mean_t(g_var) + mean_t(g_mu) per part; g_chi = g_p +
// eta g_c + c chi with c = Re(conj(g_c) (G + chi)) eta' / |chi| (through
// eta(|chi|)); g_R = conj(1 / (beta (1 - R)^2)) g_chi, or zero with R held fixed
template <typename T>
__global__ __launch_bounds__(256) void k_ccl_adj3(CcoLossArgs<T> a) {
  __shared__ double red[16];
  const int M = a.M, N = M * M, b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double bad = 0.0;
  if (n < N) {
    const int i = n / M, j = n % M;
    const T* w = a.ws + size_t(b) * kCclArrays * N;
    const size_t o = size_t(b) * N + n;
    const cx<T> z = a.chi[o], g = a.g[o];
    const T mag = sqrt(z.x * z.x + z.y * z.y);
    const T sg = T(1) / (T(1) + exp(-(mag - T(a.tau)) / T(a.delta)));
    const T eta = T(a.eta_max) * sg;
    const T deta = T(a.eta_max) * sg * (T(1) - sg) / T(a.delta);
    const T u[2] = {(T(1) + eta) * g.x, (T(1) + eta) * g.y}, p[2] = {z.x, z.y};
    T gp[2], G[2];
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const T ba = w[(kCclBA + ch) * N + n];
      gp[ch] = ba * u[ch] + T(2) * p[ch] * box_mean_t(w + (kCclT3 + ch) * N, i, j, M, a.r) +
               box_mean_t(w + (kCclT4 + ch) * N, i, j, M, a.r);
      G[ch] = ba * p[ch] + box_mean(w + (kCclB + ch) * N, i, j, M, a.r);
    }
    const T c = mag > T(0) ? (g.x * (G[0] + z.x) + g.y * (G[1] + z.y)) * deta / mag : T(0);
    const cx<T> gc{gp[0] + eta * g.x + c * z.x, gp[1] + eta * g.y + c * z.y};
    cx<T> gR{T(0), T(0)};
    if (!a.r_stopgrad) {
      const cx<T> R = a.R[o];
      const cx<T> om{T(1) - R.x, -R.y};
      const cx<T> ww = om * om;
      const T dd = T(a.beta) * norm2(ww);
      gR = cx<T>{(ww.x * gc.x - ww.y * gc.y) / dd, (ww.x * gc.y + ww.y * gc.x) / dd};
    }
    if (!(isfinite(gR.x) && isfinite(gR.y))) bad = 1.0;
    a.g[o] = gR;
  }
  const double nb = block_sum(bad, red);
  if (threadIdx.x == 0 && nb > 0.0 && a.loss) a.loss[size_t(b) * 8 + 7] = 1.0;
}

}  // namespace pdfk
