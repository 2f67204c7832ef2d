// Coupling kernels of a reconstruction measured at several frequencies: the
// contrast is one (a non-dispersive medium), so R and chi are shared while
// coefficients, currents, fields and operators are per frequency.  The
// per-frequency passes run on one handle per frequency; these kernels join
// them where the frequencies meet: the per-pixel least-squares contrast over
// all frequencies and incidences (each frequency weighted by 1/||E_inc,f||^2,
// so that R stays the exact minimiser of the summed state loss), the
// back-propagation contrast of the start value, and its line search.
#pragma once

#include "cplx.h"
#include "pixel_kernels.h"

namespace pdfk {

constexpr int kMaxFreq = 8;

// R = beta num / den from the weighted per-frequency sums of the pixel
// reductions, wsum [F][N][4] = w_f (Re num, Im num, den, sum |J|^2), or R =
// Rfix; chi = R / (beta (1 - R)); den is kept (the adjoint's regulariser part
// divides by it); lsp[tile] = sum over the tile's pixels of
// sum_f w_f sum_p |R E - beta J|^2.  Grid: ceil(N / 256) tiles of 256 pixels.
template <typename T>
__global__ __launch_bounds__(256) void k_mf_combine(const double* __restrict__ wsum, int F, int N, double beta,
                                                    const cx<T>* __restrict__ Rfix, cx<T>* __restrict__ R,
                                                    T* __restrict__ den, cx<T>* __restrict__ chi,
                                                    double* __restrict__ lsp) {
  __shared__ double red[16];
  const int n = blockIdx.x * 256 + threadIdx.x;
  double lpix = 0.0;
  if (n < N) {
    double nr = 0, ni = 0, dd = 0, jj = 0;
    for (int f = 0; f < F; ++f) {
      const double* s = wsum + (size_t(f) * N + n) * 4;
      nr += s[0];
      ni += s[1];
      dd += s[2];
      jj += s[3];
    }
    double rr, ri;
    if (Rfix) {
      rr = Rfix[n].x;
      ri = Rfix[n].y;
    } else {
      rr = beta * nr / dd;
      ri = beta * ni / dd;
      R[n] = cx<T>{T(rr), T(ri)};
    }
    lpix = (rr * rr + ri * ri) * dd - 2.0 * beta * (rr * nr + ri * ni) + beta * beta * jj;
    den[n] = T(dd);
    const double xr = 1.0 - rr, xi = -ri;
    const double q = beta * (xr * xr + xi * xi);
    chi[n] = cx<T>{T((rr * xr + ri * xi) / q), T((ri * xr - rr * xi) / q)};
  }
  const double s = block_sum(lpix, red);
  if (threadIdx.x == 0) lsp[blockIdx.x] = s;
}

template <typename T>
struct MfPairs {
  const cx<T>* J[kMaxFreq];   // [Ni][N] per frequency
  const cx<T>* E[kMaxFreq];
  double w[kMaxFreq];         // 1 / ||E_inc,f||^2
  int F, Ni, N;
};

// Back-propagation contrast over all frequencies and incidences:
// chi_0 = sum_f w_f sum_p J conj(E) / sum_f w_f sum_p |E|^2, R_0 = beta chi_0 / (beta chi_0 + 1).
template <typename T>
__global__ __launch_bounds__(256) void k_mf_bp_contrast(MfPairs<T> a, double beta, cx<T>* __restrict__ R0) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  double nr = 0, ni = 0, dd = 0;
  for (int f = 0; f < a.F; ++f) {
    double fr = 0, fi = 0, fd = 0;
    for (int p = 0; p < a.Ni; ++p) {
      const size_t idx = size_t(p) * a.N + n;
      const cx<T> j = a.J[f][idx], e = a.E[f][idx];
      fr += double(j.x) * e.x + double(j.y) * e.y;
      fi += double(j.y) * e.x - double(j.x) * e.y;
      fd += double(e.x) * e.x + double(e.y) * e.y;
    }
    nr += a.w[f] * fr;
    ni += a.w[f] * fi;
    dd += a.w[f] * fd;
  }
  const double cr = nr / dd, ci = ni / dd;
  const double ar = beta * cr, ai = beta * ci;
  const double br = ar + 1.0, bi = ai;
  const double q = br * br + bi * bi;
  R0[n] = cx<T>{T((ar * br + ai * bi) / q), T((ai * br - ar * bi) / q)};
}

// ||sum over the split-K parts||^2 of one frequency's outputs, in parts: 16
// outputs per workgroup, each summed by 16 threads (every 16th part) and
// combined in a fixed order; part[blockIdx.x] = the workgroup's sum of |x|^2.
// Grid ceil(NO / 16), 256 threads.
template <typename T>
__global__ __launch_bounds__(256) void k_mf_dnorm(const cx<T>* __restrict__ Dpart, int ntiles, int NO,
                                                  double* __restrict__ part) {
  constexpr int OUT = 16, SL = 16;
  __shared__ double sr[SL][OUT], si[SL][OUT];
  const int lo = threadIdx.x % OUT, sl = threadIdx.x / OUT;
  const int o = blockIdx.x * OUT + lo;
  double xr = 0.0, xi = 0.0;
  if (o < NO)
    for (int t = sl; t < ntiles; t += SL) {
      const cx<T> v = Dpart[size_t(t) * NO + o];
      xr += v.x;
      xi += v.y;
    }
  sr[sl][lo] = xr;
  si[sl][lo] = xi;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < OUT; ++q) {
      double ar = 0.0, ai = 0.0;
      for (int k = 0; k < SL; ++k) {
        ar += sr[k][q];
        ai += si[k][q];
      }
      s += ar * ar + ai * ai;
    }
    part[blockIdx.x] = s;
  }
}

template <typename T>
struct MfLineSearch {
  const double* dpart[kMaxFreq];  // [ndp] parts of ||G_S,f J_g||^2 per frequency (k_mf_dnorm)
  const double* lsp[kMaxFreq];    // [ntiles] sum_p |R_0 E - beta J|^2 per frequency (unweighted)
  const double* Sd[kMaxFreq];     // ||E_sca,f||^2
  const double* Ss[kMaxFreq];     // ||E_inc,f||^2
  const double* gn;               // [F] ||g_f||^2
  const cx<T>* g0[kMaxFreq];      // [Ni][K][K] gradient of L^CSI at zero per frequency
  cx<T>* alpha;                   // [F][Ni][K][K] out
  int F, ndp, ntiles, len;        // ntiles: parts of lsp, len = Ni K^2
};

// The exact line search of the summed L^CSI along -g (one workgroup):
// t* = (sum_f ||g_f||^2 / 2) / sum_f (||A_d,f g_f||^2 / S_d,f + ||A_s,f g_f||^2 / S_s,f), alpha_f = -t* g_f.
template <typename T>
__global__ __launch_bounds__(256) void k_mf_line_search(MfLineSearch<T> a) {
  __shared__ double tstar;
  const int tid = threadIdx.x;
  double q = 0.0, gsum = 0.0;
  if (tid == 0)
    for (int f = 0; f < a.F; ++f) {
      double sd = 0.0, ss = 0.0;
      for (int k = 0; k < a.ndp; ++k) sd += a.dpart[f][k];
      for (int t = 0; t < a.ntiles; ++t) ss += a.lsp[f][t];
      q += sd / a.Sd[f][0] + ss / a.Ss[f][0];
      gsum += a.gn[f];
    }
  if (tid == 0) tstar = q > 0 ? 0.5 * gsum / q : 0.0;
  __syncthreads();
  const T t = T(tstar);
  for (int f = 0; f < a.F; ++f)
    for (int e = tid; e < a.len; e += blockDim.x) {
      const cx<T> g = a.g0[f][e];
      a.alpha[size_t(f) * a.len + e] = cx<T>{-t * g.x, -t * g.y};
    }
}

}  // namespace pdfk
