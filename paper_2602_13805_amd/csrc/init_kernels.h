// Kernels of the start value (Sec. 3.1) and of the reconstruction loop.
#pragma once

#include "cplx.h"
#include "pixel_kernels.h"

namespace pdfk {

// Back-propagation scalar of one (instance, incidence) pair (grid: B * Ni):
//   v = G_S u (reduced here from the split-K parts), gamma = (v^H e)/(v^H v),
//   u <- gamma u, so that J_BP = gamma G_S^H e.
template <typename T>
__global__ __launch_bounds__(256) void k_bp_gamma(const cx<T>* Dpart, int ntiles, const cx<T>* esca,
                                                  cx<T>* u, int Ni, int Ns, int N) {
  __shared__ double red[16];
  __shared__ double gam[2];
  const int bp = blockIdx.x, b = bp / Ni, p = bp % Ni, tid = threadIdx.x;
  double nr = 0, ni = 0, dd = 0;
  for (int q = tid; q < Ns; q += blockDim.x) {
    double vr = 0, vi = 0;
    for (int t = 0; t < ntiles; ++t) {
      const cx<T> x = Dpart[((size_t(b) * ntiles + t) * Ni + p) * Ns + q];
      vr += x.x;
      vi += x.y;
    }
    const cx<T> e = esca[(size_t(b) * Ni + p) * Ns + q];
    nr += vr * e.x + vi * e.y;  // conj(v) e
    ni += vr * e.y - vi * e.x;
    dd += vr * vr + vi * vi;
  }
  const double snr = block_sum(nr, red);
  const double sni = block_sum(ni, red);
  const double sdd = block_sum(dd, red);
  if (tid == 0) {
    gam[0] = sdd > 0 ? snr / sdd : 0.0;
    gam[1] = sdd > 0 ? sni / sdd : 0.0;
  }
  __syncthreads();
  const cx<T> g{T(gam[0]), T(gam[1])};
  cx<T>* row = u + size_t(bp) * N;
  for (int n = tid; n < N; n += blockDim.x) row[n] = g * row[n];
}

// chi_0 = sum_p J conj(E) / sum_p |E|^2 and R_0 = beta chi_0 / (beta chi_0 + 1) (Eq. 7).
template <typename T>
__global__ __launch_bounds__(256) void k_bp_contrast(const cx<T>* J, const cx<T>* E, cx<T>* R0, int Ni, int N,
                                                     double beta) {
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double nr = 0, ni = 0, dd = 0;
  for (int p = 0; p < Ni; ++p) {
    const size_t idx = (size_t(b) * Ni + p) * N + n;
    const cx<T> j = J[idx], e = E[idx];
    nr += double(j.x) * e.x + double(j.y) * e.y;
    ni += double(j.y) * e.x - double(j.x) * e.y;
    dd += double(e.x) * e.x + double(e.y) * e.y;
  }
  const double cr = nr / dd, ci = ni / dd;
  // R0 = beta chi / (beta chi + 1)
  const double ar = beta * cr, ai = beta * ci;
  const double br = ar + 1.0, bi = ai;
  const double q = br * br + bi * bi;
  R0[size_t(b) * N + n] = cx<T>{T((ar * br + ai * bi) / q), T((ai * br - ar * bi) / q)};
}

// Exact line search of the quadratic L^CSI along -g (grid: B):
//   t* = (||g||^2 / 2) / (||A_d g||^2 / S_d + ||A_s g||^2 / S_s),  alpha_0 = -t* g.
template <typename T>
__global__ __launch_bounds__(256) void k_line_search(const double* lsp, const cx<T>* Dpart, int ntiles, int Ni,
                                                     int Ns, const double* gnorm, const double* Ss,
                                                     const double* Sd, const cx<T>* g0, cx<T>* alpha, int KK) {
  __shared__ double red[16];
  __shared__ double tstar;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int NO = Ni * Ns;
  double dsum = 0.0;
  for (int o = tid; o < NO; o += blockDim.x) {
    double xr = 0, xi = 0;
    for (int t = 0; t < ntiles; ++t) {
      const cx<T> v = Dpart[(size_t(b) * ntiles + t) * NO + o];
      xr += v.x;
      xi += v.y;
    }
    dsum += xr * xr + xi * xi;
  }
  const double sd = block_sum(dsum, red);
  if (tid == 0) {
    double ss = 0.0;
    for (int t = 0; t < ntiles; ++t) ss += lsp[size_t(b) * ntiles + t];
    const double q = sd / Sd[b] + ss / Ss[0];
    tstar = q > 0 ? 0.5 * gnorm[b] / q : 0.0;
  }
  __syncthreads();
  const T t = T(tstar);
  const size_t len = size_t(Ni) * KK;
  for (size_t e = tid; e < len; e += blockDim.x) {
    const cx<T> g = g0[size_t(b) * len + e];
    alpha[size_t(b) * len + e] = cx<T>{-t * g.x, -t * g.y};
  }
}

// Error bookkeeping of the reconstruction loop: lowest error so far, and
// stop updating an instance once its image error reaches its target.
__global__ void k_track_error(const double* err, const double* target, int* frozen, int* reached,
                              double* best_err, int* best_iter, const int* tstep, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (best_err && err[b] < best_err[b]) {
    best_err[b] = err[b];
    if (best_iter) best_iter[b] = tstep[b];
  }
  if (target && !frozen[b] && err[b] <= target[b]) {
    frozen[b] = 1;
    if (reached) reached[b] = tstep[b];
  }
}

// Keeps, per instance, the start with the lower total loss (loss rows of 8,
// total at index 5): alpha <- alt where loss_alt < loss_bp (grid: x over the
// len values of an instance, y over instances).
template <typename T>
__global__ void k_pick_start(cx<T>* alpha, const cx<T>* alt, const double* loss_bp, const double* loss_alt,
                             int len, int* chosen, double* loss_out) {
  const int b = blockIdx.y;
  const double lb = loss_bp[size_t(b) * 8 + 5], la = loss_alt[size_t(b) * 8 + 5];
  const bool take = la < lb;  // false for a non-finite network start
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (take && e < len) alpha[size_t(b) * len + e] = alt[size_t(b) * len + e];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (chosen) chosen[b] = take ? 1 : 0;
    if (loss_out) {
      loss_out[2 * b] = lb;
      loss_out[2 * b + 1] = la;
    }
  }
}

__global__ void k_fill_double(double* x, double v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_fill_int(int* x, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

template <typename T>
__global__ void k_fill_cx(cx<T>* x, T re, T im, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = cx<T>{re, im};
}

template <typename T>
__global__ void k_fill_zero(T* x, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = T(0);
}

// ---- the full CSI start (Sec. 3.1): conjugate gradients on the quadratic L^CSI, R fixed at R_0

// Data residual (of L^CSI, and per frequency of L^Data) d = sum over the
// split-K parts of G_S J - E_sca, per (incidence, receiver)
// output o of instance b: 16 outputs per workgroup, the parts of each summed by
// 16 threads (every 16th part) and the 16 sums added in a fixed order.
// Grid (ceil(Ni Ns / 16), B), 256 threads.
template <typename T>
__global__ __launch_bounds__(256) void k_csi_residual(const cx<T>* Dpart, int ntiles, const cx<T>* esca, cx<T>* dres,
                                                      int NO) {
  constexpr int OUT = 16, SL = 16;
  __shared__ double sr[SL][OUT], si[SL][OUT];
  const int b = blockIdx.y, lo = threadIdx.x % OUT, sl = threadIdx.x / OUT;
  const int o = blockIdx.x * OUT + lo;
  double xr = 0.0, xi = 0.0;
  if (o < NO)
    for (int t = sl; t < ntiles; t += SL) {
      const cx<T> v = Dpart[(size_t(b) * ntiles + t) * NO + o];
      xr += v.x;
      xi += v.y;
    }
  sr[sl][lo] = xr;
  si[sl][lo] = xi;
  __syncthreads();
  if (sl == 0 && o < NO) {
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < SL; ++k) {
      ar += sr[k][lo];
      ai += si[k][lo];
    }
    const cx<T> e = esca[size_t(b) * NO + o];
    dres[size_t(b) * NO + o] = cx<T>{T(ar - double(e.x)), T(ai - double(e.y))};
  }
}

// Conjugate direction p = -g + (||g||^2 / ||g_prev||^2) p (p = -g when first), the
// numerator -Re<g, p> of the exact step, and ||g||^2 kept for the next direction.
// One block per instance.
template <typename T>
__global__ __launch_bounds__(256) void k_csi_dir(const cx<T>* g, cx<T>* p, const double* gn, double* gn_prev,
                                                 double* dot, size_t len, int first) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  const double fr = (first || !(gn_prev[b] > 0.0)) ? 0.0 : gn[b] / gn_prev[b];
  const T f = T(fr);
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < len; i += blockDim.x) {
    const size_t k = size_t(b) * len + i;
    const cx<T> gv = g[k];
    cx<T> pv = cx<T>{-gv.x, -gv.y};
    if (!first) {
      const cx<T> po = p[k];
      pv = cx<T>{f * po.x - gv.x, f * po.y - gv.y};
    }
    p[k] = pv;
    acc -= double(gv.x) * pv.x + double(gv.y) * pv.y;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) {
    dot[b] = s;
    gn_prev[b] = gn[b];
  }
}

// Exact step along p: t = dot / (2 (||G_S J_p||^2 / S_d + ||R_0 E_p - beta J_p||^2 / S_s)),
// alpha += t p.  One block per instance.
template <typename T>
__global__ __launch_bounds__(256) void k_csi_step(const double* lsp, const cx<T>* Dpart, int ntiles, int Ni, int Ns,
                                                  const double* dot, const double* Ss, const double* Sd,
                                                  const cx<T>* p, cx<T>* alpha, int KK) {
  __shared__ double red[16];
  __shared__ double tstar;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int NO = Ni * Ns;
  double dsum = 0.0;
  for (int o = tid; o < NO; o += blockDim.x) {
    double xr = 0, xi = 0;
    for (int t = 0; t < ntiles; ++t) {
      const cx<T> v = Dpart[(size_t(b) * ntiles + t) * NO + o];
      xr += v.x;
      xi += v.y;
    }
    dsum += xr * xr + xi * xi;
  }
  const double sd = block_sum(dsum, red);
  if (tid == 0) {
    double ss = 0.0;
    for (int t = 0; t < ntiles; ++t) ss += lsp[size_t(b) * ntiles + t];
    const double q = sd / Sd[b] + ss / Ss[0];
    tstar = q > 0 ? 0.5 * dot[b] / q : 0.0;
  }
  __syncthreads();
  const T t = T(tstar);
  const size_t len = size_t(Ni) * KK;
  for (size_t e = tid; e < len; e += blockDim.x) {
    const size_t k = size_t(b) * len + e;
    const cx<T> a = alpha[k], d = p[k];
    alpha[k] = cx<T>{a.x + t * d.x, a.y + t * d.y};
  }
}

}  // namespace pdfk
