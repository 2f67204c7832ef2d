// Host driver of the operator-table code, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_host.py: builds the tables
// of several geometries (power-of-two and other padded sizes) and writes them
// to a binary file for comparison with the oracle, then checks that invalid
// geometries are refused.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "tables.h"

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "wb");
  if (!f) return 2;
  const int Ms[] = {8, 12, 16, 48};
  const int nis[] = {3, 4, 5, 2};
  const int nss[] = {5, 4, 7, 3};
  for (int c = 0; c < 4; ++c) {
    const int M = Ms[c], ni = nis[c], ns = nss[c];
    std::vector<double> tx(2 * ni), rx(2 * ns);
    for (int i = 0; i < ni; ++i) {
      tx[2 * i] = 2.25 * std::cos(6.283185307179586 * i / ni + 0.1);
      tx[2 * i + 1] = 2.25 * std::sin(6.283185307179586 * i / ni + 0.1);
    }
    for (int i = 0; i < ns; ++i) {
      rx[2 * i] = 2.25 * std::cos(6.283185307179586 * i / ns);
      rx[2 * i + 1] = 2.25 * std::sin(6.283185307179586 * i / ns);
    }
    pdfh::Geometry g{M, 1.5, 0.01, -0.02, 4e8, ni, ns, tx.data(), rx.data()};
    pdfh::Tables t;
    std::string err;
    if (pdfh::build_tables(g, &t, &err)) {
      std::fprintf(stderr, "build_tables failed: %s\n", err.c_str());
      return 1;
    }
    const int hdr[3] = {M, ni, ns};
    std::fwrite(hdr, sizeof(int), 3, f);
    std::fwrite(tx.data(), sizeof(double), tx.size(), f);
    std::fwrite(rx.data(), sizeof(double), rx.size(), f);
    std::fwrite(t.ghat.data(), sizeof(double) * 2, t.ghat.size(), f);
    std::fwrite(t.gs.data(), sizeof(double) * 2, t.gs.size(), f);
    std::fwrite(t.einc.data(), sizeof(double) * 2, t.einc.size(), f);
  }
  std::fclose(f);
  // invalid geometries are refused with a message
  std::vector<double> a(2, 1.0);
  for (int c = 0; c < 3; ++c) {
    pdfh::Geometry g{c == 0 ? 0 : 8, c == 1 ? -1.0 : 1.5, 0.0, 0.0, c == 2 ? 0.0 : 4e8, 1, 1, a.data(), a.data()};
    pdfh::Tables t;
    std::string err;
    if (pdfh::build_tables(g, &t, &err) == 0 || err.empty()) {
      std::fprintf(stderr, "invalid geometry %d accepted\n", c);
      return 1;
    }
  }
  std::printf("SANITIZED_OK\n");
  return 0;
}
