// Host FP64 operator tables (see tables.cpp).
#pragma once

#include <complex>
#include <functional>
#include <string>
#include <vector>

namespace pdfh {

struct Geometry {
  int M;
  double side, cx, cy, freq;
  int ni, ns;
  const double* tx;  // [ni][2]
  const double* rx;  // [ns][2]
};

struct Tables {
  bool want_ghat = true, want_gs = true, want_einc = true;
  std::vector<std::complex<double>> ghat;  // [2M][2M], unscaled FFT of the embedded kernel
  std::vector<std::complex<double>> gs;    // [ns][M*M]
  std::vector<std::complex<double>> einc;  // [ni][M*M]
  double k0 = 0.0;
  std::complex<double> cell, self;
};

int build_tables(const Geometry& g, Tables* t, std::string* err);
std::complex<double> hankel1(int n, double x);
// Runs fn(begin, end) over [0, n) split across host threads.
void parallel_for(int n, const std::function<void(int, int)>& fn);
// The same with at most max_threads threads (at most 16 in any case).
void parallel_for(int n, int max_threads, const std::function<void(int, int)>& fn);
void offset_kernel(int M, double h, double k0, std::vector<std::complex<double>>* ker);

}  // namespace pdfh
