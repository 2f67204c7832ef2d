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
#include <thread>
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

// Device allocations of one solve, stream-ordered so that concurrent solves
// on other streams are not serialised by allocation or release.
// Values of c_a H0(k0 |r_a - r_c|) for antennas a and support pixels c by
// cubic Hermite interpolation of H0^(1) between samples at multiples of dx
// (tab[2i] = H0(x_i), tab[2i+1] = H1(x_i), x_i = (i0 + i) dx, H0' = -H1).
// The nodes depend on dx only, not on the table's extent, so every value is
// the same whatever other antennas shared the table.
__global__ void k_antenna_field(const double* axy, const cx<double>* ascale, int na, const double* px,
                                const double* py, int nS, double k0, const cx<double>* tab, int i0, int nt,
                                double dx, cx<double>* out) {
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= size_t(na) * nS) return;
  const int a = int(idx / nS), c = int(idx % nS);
  const double x = k0 * hypot(axy[2 * a] - px[c], axy[2 * a + 1] - py[c]);
  const double xs = x / dx, fl = floor(xs), t = xs - fl;
  const int i = min(max(int(fl) - i0, 0), nt - 2);
  const cx<double> f0 = tab[2 * i], f1 = tab[2 * i + 2];
  const cx<double> d0{-dx * tab[2 * i + 1].x, -dx * tab[2 * i + 1].y};
  const cx<double> d1{-dx * tab[2 * i + 3].x, -dx * tab[2 * i + 3].y};
  const double u = 1.0 - t;
  const double h00 = (1.0 + 2.0 * t) * u * u, h10 = t * u * u, h01 = t * t * (3.0 - 2.0 * t), h11 = -t * t * u;
  const cx<double> v{h00 * f0.x + h10 * d0.x + h01 * f1.x + h11 * d1.x, h00 * f0.y + h10 * d0.y + h01 * f1.y + h11 * d1.y};
  out[idx] = ascale[a] * v;
}

// Stream-ordered device buffers of one solve.  The destructor first waits
// for the stream, so every copy still queued (on an early error return too)
// has finished with its host source or destination before the host vectors
// declared ahead of this object are destroyed, then releases the buffers.
struct Dev {
  hipStream_t st;
  std::vector<void*> ptrs;
  explicit Dev(hipStream_t s) : st(s) {}
  ~Dev() {
    (void)hipStreamSynchronize(st);
    for (void* p : ptrs) (void)hipFreeAsync(p, st);
    (void)hipStreamSynchronize(st);
  }
  template <typename T>
  hipError_t alloc(T** p, size_t bytes) {
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(p), bytes, st);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

// What every solve of one grid and frequency shares.
struct Shared {
  int M = 0;
  double side = 0, gx = 0, gy = 0, k0 = 0, h = 0;  // grid side and centre
  cd cell;
  std::vector<cd> ker;               // offset kernel [(2M-1)^2]
  const cx<double>* dker = nullptr;  // its device copy
  // Hankel samples for the antenna fields (null: evaluate on the host)
  const cx<double>* dtab = nullptr;  // [nt][2] H0, H1 at (i0 + i) dx
  int i0 = 0, nt = 0;
  double dx = 0.0;
};

// Hermite error about dx^4 / 384 times the fourth derivative of H0: below 1e-13 for x >= 1
constexpr double kTabDx = 2e-3;
constexpr double kTabMinX = 1.0;  // closer antennas (larger derivatives) use the host path

#define MOM_TRY(call)                                                  \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) {                                            \
      *err = std::string(#call) + ": " + hipGetErrorString(e_);        \
      return PDF_EHIP;                                                 \
    }                                                                  \
  } while (0)

// One solve: E_sca [Ni][Ns] into out; with d > 0 also the induced currents
// chi E averaged over d x d pixel blocks, [Ni][M/d][M/d], into jc.
int solve_one(const Shared& sh, const pdf_array* tx, const pdf_array* rx, const cd* eps, double tol, cd* out,
              int d, cd* jc, hipStream_t st, int host_threads, std::string* err) {
  const int M = sh.M, N = M * M, ni = tx->n, ns = rx->n;
  std::vector<int> S;
  for (int n = 0; n < N; ++n)
    if (eps[n] != cd(1.0, 0.0)) S.push_back(n);
  const int nS = int(S.size());
  const int Mc = d > 0 ? M / d : 0;
  if (jc) std::fill(jc, jc + size_t(ni) * Mc * Mc, cd(0.0));
  if (nS == 0) {
    for (int i = 0; i < ni * ns; ++i) out[i] = 0.0;
    return PDF_OK;
  }
  if (nS > 20000) {
    *err = "support larger than 20000 pixels";
    return PDF_EUNSUPPORTED;
  }
  const double k0 = sh.k0, h = sh.h;
  std::vector<int> si(nS), sj(nS);
  std::vector<cd> chi(nS), einc, gsS;
  if (!sh.dtab) {
    einc.resize(size_t(ni) * nS);
    gsS.resize(size_t(ns) * nS);
  }
  std::vector<double> xs(nS), ys(nS);
  for (int c = 0; c < nS; ++c) {
    si[c] = S[c] / M;
    sj[c] = S[c] % M;
    chi[c] = eps[S[c]] - 1.0;
    xs[c] = sh.gx - sh.side / 2.0 + (sj[c] + 0.5) * h;
    ys[c] = sh.gy - sh.side / 2.0 + (si[c] + 0.5) * h;
  }
  // incident fields and receiver operator on the support only: on the device
  // from the shared Hankel samples, else on the host
  const bool dev_fields = sh.dtab != nullptr;
  // every host array handed to an asynchronous copy is declared here, ahead of
  // the device buffers (dv), so it outlives the stream synchronisation in dv's
  // destructor on every return path
  std::vector<cd> tscale(ni), rscale(ns, sh.cell);
  std::vector<cd> mone(ni, -1.0), bnorm(ni), rho(ni), rho_old(ni, 1.0), alpha(ni, 1.0), omega(ni, 1.0), tmp(ni),
      tmp2(ni), beta(ni), nalpha(ni), nomega(ni);
  std::vector<cd> xh(jc ? size_t(ni) * nS : 0);
  for (int p = 0; p < ni; ++p)
    tscale[p] = 1.0 / std::abs(pdfh::hankel1(0, k0 * std::hypot(tx->xy[2 * p] - sh.gx, tx->xy[2 * p + 1] - sh.gy)));
  if (!dev_fields)
    pdfh::parallel_for(ni + ns, host_threads, [&](int b0, int b1) {
      for (int r = b0; r < b1; ++r) {
        const bool is_tx = r < ni;
        const double* xy = is_tx ? tx->xy + 2 * r : rx->xy + 2 * (r - ni);
        const cd scale = is_tx ? tscale[r] : sh.cell;
        cd* dst = is_tx ? &einc[size_t(r) * nS] : &gsS[size_t(r - ni) * nS];
        for (int c = 0; c < nS; ++c) dst[c] = scale * pdfh::hankel1(0, k0 * std::hypot(xy[0] - xs[c], xy[1] - ys[c]));
      }
    });

  Dev dv(st);
  cx<double> *dA, *dchi, *db, *dgs, *x, *r, *rh, *p, *v, *s, *tt, *dots, *sc1, *sc2, *dout;
  int *dsi, *dsj;
  const size_t vb = sizeof(cx<double>) * size_t(ni) * nS;
  MOM_TRY(dv.alloc(&dA, sizeof(cx<double>) * size_t(nS) * nS));
  MOM_TRY(dv.alloc(&dchi, sizeof(cx<double>) * nS));
  MOM_TRY(dv.alloc(&dsi, sizeof(int) * nS));
  MOM_TRY(dv.alloc(&dsj, sizeof(int) * nS));
  MOM_TRY(dv.alloc(&db, vb));
  MOM_TRY(dv.alloc(&dgs, sizeof(cx<double>) * size_t(ns) * nS));
  for (auto** q : {&x, &r, &rh, &p, &v, &s, &tt}) MOM_TRY(dv.alloc(q, vb));
  MOM_TRY(dv.alloc(&dots, sizeof(cx<double>) * ni * 3));
  MOM_TRY(dv.alloc(&sc1, sizeof(cx<double>) * ni));
  MOM_TRY(dv.alloc(&sc2, sizeof(cx<double>) * ni));
  MOM_TRY(dv.alloc(&dout, sizeof(cx<double>) * ni * ns));
  MOM_TRY(hipMemcpyAsync(dchi, chi.data(), sizeof(cd) * nS, hipMemcpyHostToDevice, st));
  MOM_TRY(hipMemcpyAsync(dsi, si.data(), sizeof(int) * nS, hipMemcpyHostToDevice, st));
  MOM_TRY(hipMemcpyAsync(dsj, sj.data(), sizeof(int) * nS, hipMemcpyHostToDevice, st));
  if (dev_fields) {
    double *dpx, *dpy, *daxy;
    cx<double>* dsc;
    MOM_TRY(dv.alloc(&dpx, sizeof(double) * nS));
    MOM_TRY(dv.alloc(&dpy, sizeof(double) * nS));
    MOM_TRY(dv.alloc(&daxy, sizeof(double) * 2 * (ni + ns)));
    MOM_TRY(dv.alloc(&dsc, sizeof(cx<double>) * (ni + ns)));
    MOM_TRY(hipMemcpyAsync(dpx, xs.data(), sizeof(double) * nS, hipMemcpyHostToDevice, st));
    MOM_TRY(hipMemcpyAsync(dpy, ys.data(), sizeof(double) * nS, hipMemcpyHostToDevice, st));
    MOM_TRY(hipMemcpyAsync(daxy, tx->xy, sizeof(double) * 2 * ni, hipMemcpyHostToDevice, st));
    MOM_TRY(hipMemcpyAsync(daxy + 2 * ni, rx->xy, sizeof(double) * 2 * ns, hipMemcpyHostToDevice, st));
    MOM_TRY(hipMemcpyAsync(dsc, tscale.data(), sizeof(cd) * ni, hipMemcpyHostToDevice, st));
    MOM_TRY(hipMemcpyAsync(dsc + ni, rscale.data(), sizeof(cd) * ns, hipMemcpyHostToDevice, st));
    const size_t ne = size_t(ni) * nS, nr = size_t(ns) * nS;
    hipLaunchKernelGGL(k_antenna_field, dim3((ne + 255) / 256), dim3(256), 0, st, daxy, dsc, ni, dpx, dpy, nS, k0,
                       sh.dtab, sh.i0, sh.nt, sh.dx, db);
    hipLaunchKernelGGL(k_antenna_field, dim3((nr + 255) / 256), dim3(256), 0, st, daxy + 2 * ni, dsc + ni, ns, dpx,
                       dpy, nS, k0, sh.dtab, sh.i0, sh.nt, sh.dx, dgs);
    MOM_TRY(hipGetLastError());
  } else {
    MOM_TRY(hipMemcpyAsync(db, einc.data(), vb, hipMemcpyHostToDevice, st));
    MOM_TRY(hipMemcpyAsync(dgs, gsS.data(), sizeof(cd) * gsS.size(), hipMemcpyHostToDevice, st));
  }
  const size_t nA = size_t(nS) * nS;
  hipLaunchKernelGGL(k_mom_build, dim3((nA + 255) / 256), dim3(256), 0, st, dA, sh.dker, dsi, dsj, dchi, nS, M);
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
  MOM_TRY(dv.alloc(&dpart, sizeof(cx<double>) * nv * nsplit));
  auto matvec = [&](const cx<double>* in, cx<double>* o) {
    hipLaunchKernelGGL(k_zgemm, ggrid, dim3(256), 0, st, dA, in, dpart, nS, ni, kslice);
    hipLaunchKernelGGL(k_zsum, vgrid, dim3(256), 0, st, dpart, o, nv, nsplit);
  };
  auto dot = [&](const cx<double>* a, const cx<double>* b, int slot, std::vector<cd>& hv) -> hipError_t {
    hipLaunchKernelGGL(k_zdot, dim3(ni), dim3(256), 0, st, a, b, dots + slot * ni, nS);
    hipError_t e = hipMemcpyAsync(hv.data(), dots + slot * ni, sizeof(cd) * ni, hipMemcpyDeviceToHost, st);
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
        *err = "BiCGSTAB breakdown";
        return PDF_ENONFINITE;
      }
  }
  if (it >= max_it) {
    *err = "BiCGSTAB did not converge, residual " + std::to_string(worst);
    return PDF_ENONFINITE;
  }
  hipLaunchKernelGGL(k_scatter_out, dim3(ni * ns), dim3(256), 0, st, dgs, dchi, x, dout, nS, ns);
  MOM_TRY(hipGetLastError());
  MOM_TRY(hipMemcpyAsync(out, dout, sizeof(cd) * ni * ns, hipMemcpyDeviceToHost, st));
  if (jc) MOM_TRY(hipMemcpyAsync(xh.data(), x, vb, hipMemcpyDeviceToHost, st));
  MOM_TRY(hipStreamSynchronize(st));
  if (jc) {
    // induced current chi E per fine pixel, averaged over each d x d block
    const double w = 1.0 / (double(d) * d);
    for (int q = 0; q < ni; ++q)
      for (int c = 0; c < nS; ++c)
        jc[(size_t(q) * Mc + si[c] / d) * Mc + sj[c] / d] += w * chi[c] * xh[size_t(q) * nS + c];
  }
  return PDF_OK;
}

int check_args(const pdf_grid* grid, double freq_hz, double tol) {
  if (grid->M < 1 || !(grid->side > 0) || !(freq_hz > 0) || !(tol > 0)) {
    pdf_set_global_error("invalid sizes");
    return PDF_EINVAL;
  }
  return PDF_OK;
}

// Host offset kernel and its device copy (uploaded on st, which is synchronised).
int make_shared(const pdf_grid* grid, double freq_hz, int n, const pdf_array* tx, const pdf_array* rx,
                hipStream_t st, Shared* sh, cx<double>** dker, cx<double>** dtab, std::string* err) {
  sh->M = grid->M;
  sh->side = grid->side;
  sh->gx = grid->cx;
  sh->gy = grid->cy;
  sh->k0 = 2.0 * M_PI * freq_hz / 299792458.0;
  sh->h = grid->side / grid->M;
  const double a = sh->h / std::sqrt(M_PI);
  sh->cell = cd(0.0, M_PI * sh->k0 * a / 2.0) * std::cyl_bessel_j(1.0, sh->k0 * a);
  pdfh::offset_kernel(sh->M, sh->h, sh->k0, &sh->ker);
  MOM_TRY(hipMalloc(reinterpret_cast<void**>(dker), sizeof(cx<double>) * sh->ker.size()));
  MOM_TRY(hipMemcpyAsync(*dker, sh->ker.data(), sizeof(cd) * sh->ker.size(), hipMemcpyHostToDevice, st));
  sh->dker = *dker;
  // Hankel samples covering k0 |r_a - r_c| for every antenna a and pixel centre c
  const double hd = grid->side / std::sqrt(2.0);
  double xmin = HUGE_VAL, xmax = 0.0;
  for (int i = 0; i < n; ++i)
    for (const pdf_array* arr : {&tx[i], &rx[i]})
      for (int a = 0; a < arr->n; ++a) {
        const double r = std::hypot(arr->xy[2 * a] - grid->cx, arr->xy[2 * a + 1] - grid->cy);
        xmin = std::min(xmin, sh->k0 * (r - hd));
        xmax = std::max(xmax, sh->k0 * (r + hd));
      }
  if (xmin >= kTabMinX && std::isfinite(xmax)) {
    sh->dx = kTabDx;
    sh->i0 = int(std::floor(xmin / kTabDx)) - 2;
    sh->nt = int(std::ceil(xmax / kTabDx)) + 3 - sh->i0;
    std::vector<cd> tab(2 * size_t(sh->nt));
    pdfh::parallel_for(sh->nt, [&](int b0, int b1) {
      for (int i = b0; i < b1; ++i) {
        const double x = (sh->i0 + i) * kTabDx;
        tab[2 * size_t(i)] = pdfh::hankel1(0, x);
        tab[2 * size_t(i) + 1] = pdfh::hankel1(1, x);
      }
    });
    MOM_TRY(hipMalloc(reinterpret_cast<void**>(dtab), sizeof(cx<double>) * tab.size()));
    // waited for here: tab is released at the end of this block
    MOM_TRY(hipMemcpyAsync(*dtab, tab.data(), sizeof(cd) * tab.size(), hipMemcpyHostToDevice, st));
    MOM_TRY(hipStreamSynchronize(st));
    sh->dtab = *dtab;
  }
  MOM_TRY(hipStreamSynchronize(st));
  return PDF_OK;
}

}  // namespace

extern "C" int pdf_synthesize(const pdf_grid* grid, double freq_hz, const pdf_array* tx, const pdf_array* rx,
                              const double* eps_host, double tol, double* esca_host, void* stream_v) {
  if (!grid || !tx || !rx || !tx->xy || !rx->xy || !eps_host || !esca_host || !stream_v) {
    pdf_set_global_error("null argument");
    return PDF_EINVAL;
  }
  if (int rc = check_args(grid, freq_hz, tol)) return rc;
  if (tx->n < 1 || rx->n < 1) {
    pdf_set_global_error("invalid sizes");
    return PDF_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream_v;
  Shared sh;
  cx<double>* dker = nullptr;
  cx<double>* dtab = nullptr;
  std::string err;
  int rc = make_shared(grid, freq_hz, 1, tx, rx, st, &sh, &dker, &dtab, &err);
  if (rc == PDF_OK)
    rc = solve_one(sh, tx, rx, reinterpret_cast<const cd*>(eps_host), tol, reinterpret_cast<cd*>(esca_host), 0,
                   nullptr, st, 16, &err);
  (void)hipStreamSynchronize(st);
  if (dker) (void)hipFree(dker);
  if (dtab) (void)hipFree(dtab);
  if (rc) pdf_set_global_error(err);
  return rc;
}

extern "C" int pdf_synthesize_batch(const pdf_grid* grid, double freq_hz, int32_t n, const pdf_array* tx,
                                    const pdf_array* rx, const double* eps_host, double tol, double* esca_host,
                                    int32_t coarse, double* jc_host, int32_t workers, void* stream_v) {
  if (!grid || !tx || !rx || !eps_host || !esca_host || !stream_v || (coarse > 0 && !jc_host)) {
    pdf_set_global_error("null argument");
    return PDF_EINVAL;
  }
  if (int rc = check_args(grid, freq_hz, tol)) return rc;
  if (n < 0 || coarse < 0 || (coarse > 0 && grid->M % coarse != 0)) {
    pdf_set_global_error("invalid sizes (coarse must divide M)");
    return PDF_EINVAL;
  }
  if (n == 0) return PDF_OK;
  const int ni = tx[0].n, ns = rx[0].n;
  for (int i = 0; i < n; ++i)
    if (tx[i].n != ni || rx[i].n != ns || ni < 1 || ns < 1 || !tx[i].xy || !rx[i].xy) {
      pdf_set_global_error("every instance needs the same, nonzero antenna counts");
      return PDF_EINVAL;
    }
  hipStream_t st0 = (hipStream_t)stream_v;
  Shared sh;
  cx<double>* dker = nullptr;
  cx<double>* dtab = nullptr;
  std::string err0;
  if (int rc = make_shared(grid, freq_hz, n, tx, rx, st0, &sh, &dker, &dtab, &err0)) {
    pdf_set_global_error(err0);
    if (dker) (void)hipFree(dker);
    if (dtab) (void)hipFree(dtab);
    return rc;
  }
  const int W = std::max(1, std::min({int(workers > 0 ? workers : 8), int(n), 16}));
  const int host_threads = std::max(1, 16 / W);
  const size_t N = size_t(grid->M) * grid->M;
  const int Mc = coarse > 0 ? grid->M / coarse : 0;
  std::vector<int> rcs(W, PDF_OK);
  std::vector<std::string> errs(W);
  std::vector<std::thread> th;
  for (int w = 0; w < W; ++w)
    th.emplace_back([&, w]() {
      hipStream_t st;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        rcs[w] = PDF_EHIP;
        errs[w] = "hipStreamCreateWithFlags failed";
        return;
      }
      for (int i = w; i < n && rcs[w] == PDF_OK; i += W) {
        rcs[w] = solve_one(sh, &tx[i], &rx[i], reinterpret_cast<const cd*>(eps_host) + size_t(i) * N, tol,
                           reinterpret_cast<cd*>(esca_host) + size_t(i) * ni * ns, coarse,
                           coarse > 0 ? reinterpret_cast<cd*>(jc_host) + size_t(i) * ni * Mc * Mc : nullptr,
                           st, host_threads, &errs[w]);
        if (rcs[w]) errs[w] = "instance " + std::to_string(i) + ": " + errs[w];
      }
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    });
  for (auto& t : th) t.join();
  (void)hipFree(dker);
  if (dtab) (void)hipFree(dtab);
  for (int w = 0; w < W; ++w)
    if (rcs[w]) {
      pdf_set_global_error(errs[w]);
      return rcs[w];
    }
  return PDF_OK;
}
