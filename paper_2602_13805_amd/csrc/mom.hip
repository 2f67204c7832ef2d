// FP64 method-of-moments synthesis of measured fields (Sec. 2.1, Eqs. 3-4).
//
// Only pixels where chi = eps - 1 is nonzero couple, so the state equation is
// solved exactly on that support S:
//     (I - G_D[S,S] X_S) E_S = E_inc[S],     E_sca = G_S[:,S] X_S E_S,
// with G_D[S,S] gathered from the translation-invariant offset kernel.  The
// dense system is solved for all incidences at once by BiCGSTAB, whose matvec
// is a tiled complex FP64 GEMM on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/pdf.h"
#include "cplx.h"
#include "pixel_kernels.h"
#include "handle.h"
#include "tables.h"

using namespace pdfk;
using cd = std::complex<double>;

namespace {


__global__ void k_mom_build(cx<double>* A, const cx<double>* ker, const int* si, const int* sj,
                            const cx<double>* chi, int nS, int M) {
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= size_t(nS) * nS) return;
  const int a = int(idx / nS), c = int(idx % nS);
  const int W = 2 * M - 1;
  const cx<double> g = ker[size_t(si[a] - si[c] + M - 1) * W + (sj[a] - sj[c] + M - 1)];
  cx<double> v = g * chi[c];
  v.x = -v.x;
  v.y = -v.y;
  if (a == c) v.x += 1.0;
  A[idx] = v;
}

// Partial products of Y[p][a] = sum_c A[a][c] X[p][c] (A [n][n] row-major,
// X, Y [nrhs][n]) over the column slice s of the grid's y dimension:
// part[s][p][a].  Block: 64 rows x 64 right-hand sides, 256 threads, each
// 4 x 4 outputs; the slices are summed in fixed order by k_zsum.
constexpr int TBM = 64, TBN = 64, TBK = 16;
__global__ __launch_bounds__(256) void k_zgemm(const cx<double>* __restrict__ A, const cx<double>* __restrict__ X,
                                               cx<double>* __restrict__ part, int n, int nrhs, int kslice) {
  __shared__ cx<double> As[TBK][TBM + 1];
  __shared__ cx<double> Xs[TBK][TBN + 1];
  const int a0 = blockIdx.x * TBM, s = blockIdx.y;
  const int c_begin = s * kslice, c_end = min(n, c_begin + kslice);
  const int tid = threadIdx.x, ta = tid % 16, tp = tid / 16;
  cx<double> acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = cx<double>{0.0, 0.0};
  for (int c0 = c_begin; c0 < c_end; c0 += TBK) {
    for (int e = tid; e < TBM * TBK; e += 256) {
      const int r = e / TBK, k = e % TBK;
      const int a = a0 + r, c = c0 + k;
      As[k][r] = (a < n && c < c_end) ? A[size_t(a) * n + c] : cx<double>{0.0, 0.0};
    }
    for (int e = tid; e < TBN * TBK; e += 256) {
      const int r = e / TBK, k = e % TBK;
      const int c = c0 + k;
      Xs[k][r] = (r < nrhs && c < c_end) ? X[size_t(r) * n + c] : cx<double>{0.0, 0.0};
    }
    __syncthreads();
    for (int k = 0; k < TBK; ++k) {
      cx<double> av[4], xv[4];
      for (int i = 0; i < 4; ++i) av[i] = As[k][ta + 16 * i];
      for (int j = 0; j < 4; ++j) xv[j] = Xs[k][tp + 16 * j];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = acc[i][j] + av[i] * xv[j];
    }
    __syncthreads();
  }
  cx<double>* out = part + size_t(s) * nrhs * n;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + ta + 16 * i, p = tp + 16 * j;
      if (a < n && p < nrhs) out[size_t(p) * n + a] = acc[i][j];
    }
}

// Y = sum over the S slices of part, in slice order.
__global__ void k_zsum(const cx<double>* part, cx<double>* Y, size_t len, int S) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= len) return;
  cx<double> s = part[i];
  for (int k = 1; k < S; ++k) s = s + part[size_t(k) * len + i];
  Y[i] = s;
}

// out[p] = sum_c conj(X[p][c]) Y[p][c]   (one block per right-hand side)
__global__ __launch_bounds__(256) void k_zdot(const cx<double>* X, const cx<double>* Y, cx<double>* out, int n) {
  __shared__ double red[16];
  const int p = blockIdx.x;
  double re = 0, im = 0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const cx<double> x = X[size_t(p) * n + c], y = Y[size_t(p) * n + c];
    re += x.x * y.x + x.y * y.y;
    im += x.x * y.y - x.y * y.x;
  }
  const double sr = block_sum(re, red);
  const double si = block_sum(im, red);
  if (threadIdx.x == 0) out[p] = cx<double>{sr, si};
}

// Z[p] = X[p] + s1[p] * Y[p] + s2[p] * W[p]   (W may be null)
__global__ void k_zaxpy2(cx<double>* Z, const cx<double>* X, const cx<double>* Y, const cx<double>* s1,
                         const cx<double>* W, const cx<double>* s2, int n, int nrhs) {
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= size_t(n) * nrhs) return;
  const int p = int(idx / n);
  cx<double> z = X[idx] + s1[p] * Y[idx];
  if (W) z = z + s2[p] * W[idx];
  Z[idx] = z;
}

// E_sca[p][q] = sum_c G_S[q][c] chi[c] X[p][c]   (one block per (p, q))
__global__ __launch_bounds__(256) void k_scatter_out(const cx<double>* gsS, const cx<double>* chi,
                                                     const cx<double>* X, cx<double>* out, int n, int ns) {
  __shared__ double red[16];
  const int p = blockIdx.x / ns, q = blockIdx.x % ns;
  double re = 0, im = 0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const cx<double> v = gsS[size_t(q) * n + c] * (chi[c] * X[size_t(p) * n + c]);
    re += v.x;
    im += v.y;
  }
  const double sr = block_sum(re, red);
  const double si = block_sum(im, red);
  if (threadIdx.x == 0) out[blockIdx.x] = cx<double>{sr, si};
}

struct Dev {
  std::vector<void*> ptrs;
  ~Dev() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  hipError_t alloc(T** p, size_t bytes) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

}  // namespace

#define MOM_TRY(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      pdf_set_global_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return PDF_EHIP;                                                             \
    }                                                                              \
  } while (0)

extern "C" int pdf_synthesize(const pdf_grid* grid, double freq_hz, const pdf_array* tx, const pdf_array* rx,
                              const double* eps_host, double tol, double* esca_host, void* stream_v) {
  if (!grid || !tx || !rx || !tx->xy || !rx->xy || !eps_host || !esca_host || !stream_v) {
    pdf_set_global_error("null argument");
    return PDF_EINVAL;
  }
  if (grid->M < 1 || !(grid->side > 0) || !(freq_hz > 0) || tx->n < 1 || rx->n < 1 || !(tol > 0)) {
    pdf_set_global_error("invalid sizes");
    return PDF_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream_v;
  const int M = grid->M, N = M * M, ni = tx->n, ns = rx->n;
  const cd* eps = reinterpret_cast<const cd*>(eps_host);
  std::vector<int> S;
  for (int n = 0; n < N; ++n)
    if (eps[n] != cd(1.0, 0.0)) S.push_back(n);
  cd* out = reinterpret_cast<cd*>(esca_host);
  const int nS = int(S.size());
  if (nS == 0) {
    for (int i = 0; i < ni * ns; ++i) out[i] = 0.0;
    return PDF_OK;
  }
  if (nS > 20000) {
    pdf_set_global_error("support larger than 20000 pixels");
    return PDF_EUNSUPPORTED;
  }
  const double k0 = 2.0 * M_PI * freq_hz / 299792458.0;
  const double h = grid->side / M;
  const double a = h / std::sqrt(M_PI);
  const cd cell = cd(0.0, M_PI * k0 * a / 2.0) * std::cyl_bessel_j(1.0, k0 * a);
  std::vector<cd> ker;
  pdfh::offset_kernel(M, h, k0, &ker);
  std::vector<int> si(nS), sj(nS);
  std::vector<cd> chi(nS), einc(size_t(ni) * nS), gsS(size_t(ns) * nS);
  std::vector<double> xs(nS), ys(nS);
  for (int c = 0; c < nS; ++c) {
    si[c] = S[c] / M;
    sj[c] = S[c] % M;
    chi[c] = eps[S[c]] - 1.0;
    xs[c] = grid->cx - grid->side / 2.0 + (sj[c] + 0.5) * h;
    ys[c] = grid->cy - grid->side / 2.0 + (si[c] + 0.5) * h;
  }
  // incident fields and receiver operator on the support only
  pdfh::parallel_for(ni + ns, [&](int b0, int b1) {
    for (int r = b0; r < b1; ++r) {
      const bool is_tx = r < ni;
      const double* xy = is_tx ? tx->xy + 2 * r : rx->xy + 2 * (r - ni);
      cd scale = cell;
      if (is_tx) scale = 1.0 / std::abs(pdfh::hankel1(0, k0 * std::hypot(xy[0] - grid->cx, xy[1] - grid->cy)));
      cd* dst = is_tx ? &einc[size_t(r) * nS] : &gsS[size_t(r - ni) * nS];
      for (int c = 0; c < nS; ++c) dst[c] = scale * pdfh::hankel1(0, k0 * std::hypot(xy[0] - xs[c], xy[1] - ys[c]));
    }
  });

  Dev d;
  cx<double> *dA, *dker, *dchi, *db, *dgs, *x, *r, *rh, *p, *v, *s, *tt, *dots, *sc1, *sc2, *dout;
  int *dsi, *dsj;
  const size_t vb = sizeof(cx<double>) * size_t(ni) * nS;
  MOM_TRY(d.alloc(&dA, sizeof(cx<double>) * size_t(nS) * nS));
  MOM_TRY(d.alloc(&dker, sizeof(cx<double>) * ker.size()));
  MOM_TRY(d.alloc(&dchi, sizeof(cx<double>) * nS));
  MOM_TRY(d.alloc(&dsi, sizeof(int) * nS));
  MOM_TRY(d.alloc(&dsj, sizeof(int) * nS));
  MOM_TRY(d.alloc(&db, vb));
  MOM_TRY(d.alloc(&dgs, sizeof(cx<double>) * gsS.size()));
  for (auto** q : {&x, &r, &rh, &p, &v, &s, &tt}) MOM_TRY(d.alloc(q, vb));
  MOM_TRY(d.alloc(&dots, sizeof(cx<double>) * ni * 3));
  MOM_TRY(d.alloc(&sc1, sizeof(cx<double>) * ni));
  MOM_TRY(d.alloc(&sc2, sizeof(cx<double>) * ni));
  MOM_TRY(d.alloc(&dout, sizeof(cx<double>) * ni * ns));
  MOM_TRY(hipMemcpyAsync(dker, ker.data(), sizeof(cd) * ker.size(), hipMemcpyHostToDevice, st));
  MOM_TRY(hipMemcpyAsync(dchi, chi.data(), sizeof(cd) * nS, hipMemcpyHostToDevice, st));
  MOM_TRY(hipMemcpyAsync(dsi, si.data(), sizeof(int) * nS, hipMemcpyHostToDevice, st));
  MOM_TRY(hipMemcpyAsync(dsj, sj.data(), sizeof(int) * nS, hipMemcpyHostToDevice, st));
  MOM_TRY(hipMemcpyAsync(db, einc.data(), vb, hipMemcpyHostToDevice, st));
  MOM_TRY(hipMemcpyAsync(dgs, gsS.data(), sizeof(cd) * gsS.size(), hipMemcpyHostToDevice, st));
  const size_t nA = size_t(nS) * nS;
  hipLaunchKernelGGL(k_mom_build, dim3((nA + 255) / 256), dim3(256), 0, st, dA, dker, dsi, dsj, dchi, nS, M);
  MOM_TRY(hipGetLastError());

  // split the inner dimension so that about a thousand workgroups run
  const int rblocks = (nS + TBM - 1) / TBM;
  int nsplit = (1024 + rblocks - 1) / rblocks;
  nsplit = std::max(1, std::min(nsplit, (nS + TBK - 1) / TBK));
  const int kslice = (((nS + nsplit - 1) / nsplit) + TBK - 1) / TBK * TBK;
  nsplit = (nS + kslice - 1) / kslice;
  const dim3 ggrid(rblocks, nsplit);
  const size_t nv = size_t(ni) * nS;
  const dim3 vgrid((nv + 255) / 256);
  cx<double>* dpart;
  MOM_TRY(d.alloc(&dpart, sizeof(cx<double>) * nv * nsplit));
  auto matvec = [&](const cx<double>* in, cx<double>* o) {
    hipLaunchKernelGGL(k_zgemm, ggrid, dim3(256), 0, st, dA, in, dpart, nS, ni, kslice);
    hipLaunchKernelGGL(k_zsum, vgrid, dim3(256), 0, st, dpart, o, nv, nsplit);
  };
  auto dot = [&](const cx<double>* a, const cx<double>* b, int slot, std::vector<cd>& h) -> hipError_t {
    hipLaunchKernelGGL(k_zdot, dim3(ni), dim3(256), 0, st, a, b, dots + slot * ni, nS);
    hipError_t e = hipMemcpyAsync(h.data(), dots + slot * ni, sizeof(cd) * ni, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  };
  auto axpy2 = [&](cx<double>* z, const cx<double>* a, const cx<double>* b, const std::vector<cd>& s1,
                   const cx<double>* w, const std::vector<cd>& s2) -> hipError_t {
    hipError_t e = hipMemcpyAsync(sc1, s1.data(), sizeof(cd) * ni, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    if (w) {
      e = hipMemcpyAsync(sc2, s2.data(), sizeof(cd) * ni, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_zaxpy2, vgrid, dim3(256), 0, st, z, a, b, sc1, w, sc2, nS, ni);
    return hipGetLastError();
  };
  std::vector<cd> one(ni, 1.0), mone(ni, -1.0), bnorm(ni), rho(ni), rho_old(ni, 1.0), alpha(ni, 1.0),
      omega(ni, 1.0), tmp(ni), tmp2(ni), beta(ni), nalpha(ni), nomega(ni);
  std::vector<bool> conv(ni, false);
  // x0 = E_inc, r0 = b - A x0, r_hat = r0
  MOM_TRY(hipMemcpyAsync(x, db, vb, hipMemcpyDeviceToDevice, st));
  matvec(x, v);
  MOM_TRY(axpy2(r, db, v, mone, nullptr, mone));
  MOM_TRY(hipMemcpyAsync(rh, r, vb, hipMemcpyDeviceToDevice, st));
  MOM_TRY(hipMemsetAsync(p, 0, vb, st));
  MOM_TRY(hipMemsetAsync(v, 0, vb, st));
  MOM_TRY(dot(db, db, 0, bnorm));
  int it = 0;
  double worst = 1.0;
  const int max_it = 1000;
  for (; it < max_it; ++it) {
    MOM_TRY(dot(rh, r, 0, rho));
    for (int q = 0; q < ni; ++q) {
      beta[q] = conv[q] ? 0.0 : (rho[q] / rho_old[q]) * (alpha[q] / omega[q]);
      tmp[q] = -omega[q] * beta[q];
    }
    // p = r + beta p - beta omega v
    MOM_TRY(axpy2(p, r, p, beta, v, tmp));
    matvec(p, v);
    MOM_TRY(dot(rh, v, 1, tmp2));
    for (int q = 0; q < ni; ++q) {
      alpha[q] = conv[q] ? 0.0 : rho[q] / tmp2[q];
      nalpha[q] = -alpha[q];
    }
    MOM_TRY(axpy2(s, r, v, nalpha, nullptr, nalpha));  // s = r - alpha v
    matvec(s, tt);
    MOM_TRY(dot(tt, s, 1, tmp));
    MOM_TRY(dot(tt, tt, 2, tmp2));
    for (int q = 0; q < ni; ++q) {
      omega[q] = (conv[q] || std::abs(tmp2[q]) == 0.0) ? 0.0 : tmp[q] / tmp2[q];
      nomega[q] = -omega[q];
    }
    MOM_TRY(axpy2(x, x, p, alpha, s, omega));   // x += alpha p + omega s
    MOM_TRY(axpy2(r, s, tt, nomega, nullptr, nomega));  // r = s - omega t
    MOM_TRY(dot(r, r, 2, tmp));
    worst = 0.0;
    for (int q = 0; q < ni; ++q) {
      const double rel = std::sqrt(std::abs(tmp[q]) / std::abs(bnorm[q]));
      if (rel < tol) conv[q] = true;
      worst = std::max(worst, conv[q] ? 0.0 : rel);
      rho_old[q] = rho[q];  // converged columns get alpha = omega = 0 from now on
    }
    bool all = true;
    for (int q = 0; q < ni; ++q) all = all && conv[q];
    if (all) break;
    for (int q = 0; q < ni; ++q)
      if (!conv[q] && std::abs(omega[q]) == 0.0) {
        pdf_set_global_error("BiCGSTAB breakdown");
        return PDF_ENONFINITE;
      }
  }
  if (it >= max_it) {
    pdf_set_global_error("BiCGSTAB did not converge, residual " + std::to_string(worst));
    return PDF_ENONFINITE;
  }
  hipLaunchKernelGGL(k_scatter_out, dim3(ni * ns), dim3(256), 0, st, dgs, dchi, x, dout, nS, ns);
  MOM_TRY(hipGetLastError());
  MOM_TRY(hipMemcpyAsync(out, dout, sizeof(cd) * ni * ns, hipMemcpyDeviceToHost, st));
  MOM_TRY(hipStreamSynchronize(st));
  return PDF_OK;
}
