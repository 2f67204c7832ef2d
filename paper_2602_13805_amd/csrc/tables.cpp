// FP64 operator tables of one measurement geometry, on the host.
//
// Circular-cell method of moments for the 2-D TM Lippmann-Schwinger equation
// (Sec. 2.1, Eqs. 1-4), time dependence exp(-i w t): a square pixel of side h
// is replaced by the disc of equal area, radius a = h / sqrt(pi).  The cell
// integrals of k0^2 (i/4) H0^(1)(k0 |r - r'|) are
//   outside the cell:  (i pi k0 a / 2) J1(k0 a) H0(k0 rho)
//   own cell:          (i pi k0 a / 2) H1(k0 a) - 1
// The line source of transmitter p is c_p H0(k0 |r - r_p|) with
// c_p = 1 / |H0(k0 |r_p - centre|)|.
#include <cmath>
#include <complex>
#include <string>
#include <algorithm>
#include <functional>
#include <thread>
#include <vector>

#include "tables.h"

namespace pdfh {

using cd = std::complex<double>;

cd hankel1(int n, double x) { return cd(std::cyl_bessel_j(double(n), x), std::cyl_neumann(double(n), x)); }

void parallel_for(int n, const std::function<void(int, int)>& fn) { parallel_for(n, 16, fn); }

void parallel_for(int n, int max_threads, const std::function<void(int, int)>& fn) {
  int nt = int(std::thread::hardware_concurrency());
  nt = std::max(1, std::min(nt, std::min(16, max_threads)));
  nt = std::min(nt, std::max(1, n / 64));
  if (nt <= 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int a = t * chunk, b = std::min(n, a + chunk);
    if (a < b) th.emplace_back(fn, a, b);
  }
  for (auto& x : th) x.join();
}

// In-place radix-2 FFT (forward, exp(-2 pi i jk / n)) of length n = 2^m, stride s.
static void fft_pow2(cd* x, int n, int s) {
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i * s], x[j * s]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const double ang = -2.0 * M_PI / len;
    for (int i = 0; i < n; i += len) {
      for (int k = 0; k < len / 2; ++k) {
        const cd w(std::cos(ang * k), std::sin(ang * k));
        const cd u = x[(i + k) * s], v = x[(i + k + len / 2) * s] * w;
        x[(i + k) * s] = u + v;
        x[(i + k + len / 2) * s] = u - v;
      }
    }
  }
}

// Direct DFT along one axis (any length), used when n is not a power of two.
static void dft_any(cd* x, int n, int s) {
  std::vector<cd> y(n);
  for (int k = 0; k < n; ++k) {
    cd acc = 0.0;
    for (int j = 0; j < n; ++j) acc += x[j * s] * std::polar(1.0, -2.0 * M_PI * double(j) * k / n);
    y[k] = acc;
  }
  for (int k = 0; k < n; ++k) x[k * s] = y[k];
}

static void fft2(std::vector<cd>& a, int P) {
  const bool pow2 = (P & (P - 1)) == 0;
  for (int r = 0; r < P; ++r) pow2 ? fft_pow2(&a[size_t(r) * P], P, 1) : dft_any(&a[size_t(r) * P], P, 1);
  for (int c = 0; c < P; ++c) pow2 ? fft_pow2(&a[c], P, P) : dft_any(&a[c], P, P);
}

int build_tables(const Geometry& g, Tables* t, std::string* err) {
  const int M = g.M;
  if (M < 1 || !(g.side > 0) || !(g.freq > 0)) {
    *err = "invalid grid or frequency";
    return -1;
  }
  const double k0 = 2.0 * M_PI * g.freq / 299792458.0;
  const double h = g.side / M;
  const double a = h / std::sqrt(M_PI);
  const cd cell = cd(0.0, M_PI * k0 * a / 2.0) * std::cyl_bessel_j(1.0, k0 * a);
  const cd self = cd(0.0, M_PI * k0 * a / 2.0) * hankel1(1, k0 * a) - 1.0;
  const int N = M * M, P = 2 * M;
  auto px = [&](int j) { return g.cx - g.side / 2.0 + (j + 0.5) * h; };
  auto py = [&](int i) { return g.cy - g.side / 2.0 + (i + 0.5) * h; };

  if (t->want_ghat) {
    // kernel of offset (di, dj) placed at (di mod P, dj mod P); index M stays zero
    std::vector<cd> emb(size_t(P) * P, cd(0.0, 0.0));
    for (int di = -(M - 1); di <= M - 1; ++di) {
      for (int dj = -(M - 1); dj <= M - 1; ++dj) {
        cd v;
        if (di == 0 && dj == 0) {
          v = self;
        } else {
          const double rho = h * std::sqrt(double(di) * di + double(dj) * dj);
          v = cell * hankel1(0, k0 * rho);
        }
        emb[size_t((di + P) % P) * P + (dj + P) % P] = v;
      }
    }
    fft2(emb, P);
    t->ghat = std::move(emb);
  }
  if (t->want_gs) {
    t->gs.assign(size_t(g.ns) * N, cd());
    parallel_for(g.ns * M, [&](int a, int b) {
      for (int r = a; r < b; ++r) {
        const int q = r / M, i = r % M;
        for (int j = 0; j < M; ++j) {
          const double d = std::hypot(g.rx[2 * q] - px(j), g.rx[2 * q + 1] - py(i));
          t->gs[size_t(q) * N + i * M + j] = cell * hankel1(0, k0 * d);
        }
      }
    });
  }
  if (t->want_einc) {
    t->einc.assign(size_t(g.ni) * N, cd());
    parallel_for(g.ni * M, [&](int a, int b) {
      for (int r = a; r < b; ++r) {
        const int p = r / M, i = r % M;
        const double rc = std::hypot(g.tx[2 * p] - g.cx, g.tx[2 * p + 1] - g.cy);
        const double c = 1.0 / std::abs(hankel1(0, k0 * rc));
        for (int j = 0; j < M; ++j) {
          const double d = std::hypot(g.tx[2 * p] - px(j), g.tx[2 * p + 1] - py(i));
          t->einc[size_t(p) * N + i * M + j] = c * hankel1(0, k0 * d);
        }
      }
    });
  }
  t->k0 = k0;
  t->cell = cell;
  t->self = self;
  return 0;
}

// G_D as a function of the pixel offset, [2M-1][2M-1] with index (di+M-1, dj+M-1).
void offset_kernel(int M, double h, double k0, std::vector<cd>* ker) {
  const double a = h / std::sqrt(M_PI);
  const cd cell = cd(0.0, M_PI * k0 * a / 2.0) * std::cyl_bessel_j(1.0, k0 * a);
  const cd self = cd(0.0, M_PI * k0 * a / 2.0) * hankel1(1, k0 * a) - 1.0;
  const int W = 2 * M - 1;
  ker->assign(size_t(W) * W, cd());
  // the kernel depends on |offset| only: evaluate one quadrant and mirror it
  parallel_for(M, [&](int a, int b) {
    for (int di = a; di < b; ++di)
      for (int dj = 0; dj < M; ++dj) {
        cd v = self;
        if (di != 0 || dj != 0) v = cell * hankel1(0, k0 * h * std::sqrt(double(di) * di + double(dj) * dj));
        for (int si : {-1, 1})
          for (int sj : {-1, 1}) (*ker)[size_t(si * di + M - 1) * W + (sj * dj + M - 1)] = v;
      }
  });
}

}  // namespace pdfh
