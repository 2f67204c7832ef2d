// Per-incidence fused kernels: basis synthesis, the 2x-padded FFT convolution
// with the domain operator, the CIE bracket, and the adjoint pass with the
// basis analysis and Adam.  One workgroup owns one (instance, incidence) pair
// and keeps the whole padded 2M x 2M spectrum in LDS.
#pragma once

#include "cplx.h"
#include "fft_lds.h"

namespace pdfk {

template <typename T, int M_>
struct ConvCfg {
  static constexpr int M = M_;
  static constexpr int P = 2 * M;
  static constexpr int N = M * M;
  // The tile holds the M stored rows of the padded P x P grid (row stride
  // P + 1); rows M..P-1 are zero padding and are never stored: the column
  // phase works on the M stored entries of each column (see col_conv).
  using TileL = Tile<P>;
  // M = 48 (P = 96 = 3 * 32) takes radix-12 / radix-3 passes: every
  // per-thread element count carries the factor 3
  static constexpr bool TRI = M % 3 == 0;
  static constexpr int NT = M >= 96 ? 768 : (M >= 64 ? 512 : (TRI ? 384 : (M >= 32 ? 256 : 64)));
  static constexpr int EPT_M = TRI ? 12 : 8;                                     // length-M transforms (basis), workgroup-wide
  static constexpr int EPT_R = M >= 96 ? 24 : (TRI ? 12 : (M >= 64 ? 16 : 8));  // length-P transforms along rows, workgroup-wide
  static constexpr int EPT_C = M >= 96 ? 24 : (TRI ? 12 : (M >= 64 ? 16 : 8));  // length-M column chains, wave-local
  static constexpr int PPT = N / NT;              // pixels owned per thread
  static_assert(N % NT == 0, "pixel ownership must be exact");
  static_assert(P >= 16, "the column phase needs P >= 16");
  static constexpr size_t LDS_BYTES = sizeof(cx<T>) * (size_t(M) * TileL::LD + P);
  // waves per SIMD the register allocation must allow: as many as the
  // workgroups that fit one CU's 160 KB of LDS bring (two 512-thread FP32
  // workgroups at M = 64 need four; one 768-thread workgroup at M = 96,
  // three), at most four in FP32 and two in FP64
  static constexpr int lds_waves(size_t bytes) {
    const int w = int((160 * 1024) / bytes) * (NT / 64) / 4;
    const int cap = sizeof(T) == 4 ? 4 : 2;
    return w < 1 ? 1 : (w > cap ? cap : w);
  }
  static constexpr int WPE = lds_waves(LDS_BYTES);
  // the adjoint keeps g_J (PPT values per thread) through the convolution; at
  // M = 64 in FP32 the first GJ_LDS of them wait in LDS after the twiddles
  // (12 KB, still two workgroups per CU), which keeps the kernel within its
  // 128 registers
  static constexpr int GJ_LDS = (M == 64 && sizeof(T) == 4) ? 3 : 0;
  static constexpr size_t ADJ_LDS_BYTES = LDS_BYTES + sizeof(cx<T>) * size_t(GJ_LDS) * NT;
  // The second plan (PP) stores all 2M rows: the row passes then alternate
  // between rows 0..M-1 and M..2M-1 (BOT), one barrier per pass instead of
  // two, at twice the LDS (at M = 64 in FP32: one workgroup per CU, so four
  // waves per SIMD are not needed and the adjoint keeps all of g_J in
  // registers).  Both plans compute every value in the same order.
  static constexpr int BOT = M * TileL::LD;
  static constexpr size_t lds(bool pp) { return pp ? sizeof(cx<T>) * (size_t(2 * M) * TileL::LD + P) : LDS_BYTES; }
  static constexpr size_t adj_lds(bool pp) { return pp ? lds(true) : ADJ_LDS_BYTES; }
  static constexpr int wpe(bool pp) { return pp ? lds_waves(lds(true)) : WPE; }
  static constexpr int gj_lds(bool pp) { return pp ? 0 : GJ_LDS; }
  static constexpr size_t fwd_lds(bool pp, bool) { return lds(pp); }
  using Rows = Vecs<P, M, true>;                 // the M stored rows, elements along a row
  using Cols = Vecs<P, P, false, false, true>;   // all P columns (their M stored entries), wave-local
  using RowsM = Vecs<P, M, true>;                // length-M rows of the top-left M x M block
  using ColsM = Vecs<P, M, false>;
  using ModeRows = Vecs<P, M, true, true>;       // the K rows / columns of the kept modes
  using ModeCols = Vecs<P, M, false, true>;
};

// Column phase of the convolution, in place on all P columns of the M x P
// tile.  For a column with stored entries x (the padded entries M..P-1 are
// zero) the phase computes y = crop_M(IFFT_P(ghat[., c] FFT_P(pad(x)))).  The
// even and odd frequencies of the padded transform are FFT_M(x) and
// FFT_M(x w) with w[n] = exp(-2 pi i n / P), and the cropped inverse splits
// the same way, so
//   y[n] = IFFT_M(ghat[2k, c] FFT_M(x))[n] + conj(w[n]) IFFT_M(ghat[2k+1, c] FFT_M(x w))[n]:
// two length-M chains per column instead of one length-P transform, and no
// storage for the padded half.  Each wavefront owns whole columns; x and the
// first chain's result stay in registers while each chain exchanges through
// the column's own M entries.  A chain's forward last pass and inverse first
// pass share their registers, so the spectrum is applied in registers.
// The adjoint uses conj(ghat).
// BANDED: the tile's columns hold a permuted spectrum (the band-limited
// forward path below): column c < M is spectrum column 2c + 1, column M + j
// (j < ncols - M) is spectrum column 2 wrap(kmin + j); columns from ncols on
// are skipped.  Otherwise column c is spectrum column c and all P are done.
// The two chains of every column of the wave-local set `cols` (EPT elements
// per thread, NT threads); spec_col(v) is the spectrum column of vector v.
// Ends with each wavefront's own columns written back (no workgroup barrier).
template <typename T, int M, int EPT, int NT, class V, class SpecCol>
__device__ __forceinline__ void col_chains(cx<T>* buf, const cx<T>* tw, const cx<T>* ghat, bool adjoint, const V& cols,
                                           const SpecCol& spec_col) {
  constexpr int P = 2 * M;
  using F = Fft<T, M, EPT, NT, V, 2>;                     // tw[2k] = exp(-2 pi i k / M)
  constexpr int R1 = F::radix(1), R2 = M / R1;            // forward radices R1 then R2, inverse R2 then R1
  static_assert(R2 == 1 || (R2 <= 16 && EPT % R2 == 0), "a chain takes one or two passes");
  const F f{buf, tw, cols};
  typename F::Regs x;
  f.assign(x);
  f.template load<R1, 1, -1, R1>(x, NoLoad());  // butterfly j holds elements j + (M / R1) r
  // output position of register (q, u, r) after the chain's last (inverse) pass
  auto out_pos = [&](int q, int u, int r) {
    const int j = x.t[q] + u * F::TPV;
    if constexpr (R2 == 1)
      return r;
    else
      return (j / R2) * R2 * R1 + (j % R2) + r * R2;
  };
  // spectrum of the chain's frequency k = j + NSOUT r (row 2k + c of ghat) on the registers of butterfly j
  auto mul_ghat = [&](typename F::Regs& g, int c, auto rc, int NSOUT) {
    constexpr int R = decltype(rc)::value;
#pragma unroll
    for (int q = 0; q < F::UPT; ++q) {
      if (!g.act[q]) continue;
#pragma unroll
      for (int u = 0; u < EPT / R; ++u) {
        const int j = g.t[q] + u * F::TPV;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cx<T> w = ghat[(2 * (j + r * NSOUT) + c) * P + spec_col(g.vec[q])];
          if (adjoint) w.y = -w.y;
          g.v[q][u * R + r] = g.v[q][u * R + r] * w;
        }
      }
    }
  };
  cx<T> acc[F::UPT][EPT];
  static_for<2>([&](auto cc) {
    constexpr int c = decltype(cc)::value;  // 0: even frequencies, 1: odd
    F::sync();  // every lane's reads of the column are done before it is overwritten
    typename F::Regs g = x;
    if constexpr (c == 1) {  // the odd chain transforms x w
#pragma unroll
      for (int q = 0; q < F::UPT; ++q) {
        if (!g.act[q]) continue;
#pragma unroll
        for (int u = 0; u < EPT / R1; ++u) {
          const int j = g.t[q] + u * F::TPV;
#pragma unroll
          for (int r = 0; r < R1; ++r) g.v[q][u * R1 + r] = g.v[q][u * R1 + r] * tw[j + r * (M / R1)];
        }
      }
    }
    if constexpr (R2 == 1) {
      f.template compute<R1, -1, R1, R1>(g);
      mul_ghat(g, c, std::integral_constant<int, R1>{}, 1);
      f.template compute<R1, +1, R1, R1>(g);
    } else {
      f.template compute<R1, -1, R1, R1>(g);
      f.template store<R1, 1, R1>(g);
      F::sync();
      f.template load<R2, R1, -1, R2>(g, NoLoad());
      f.template compute<R2, -1, R2, R2>(g);
      mul_ghat(g, c, std::integral_constant<int, R2>{}, R1);
      f.template compute<R2, +1, R2, R2>(g);
      F::sync();
      f.template store<R2, 1, R2>(g);
      F::sync();
      f.template load<R1, R2, +1, R1>(g, NoLoad());
      f.template compute<R1, +1, R1, R1>(g);
    }
    if constexpr (c == 0) {
#pragma unroll
      for (int q = 0; q < F::UPT; ++q)
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[q][e] = g.v[q][e];
    } else {
      F::sync();
#pragma unroll
      for (int q = 0; q < F::UPT; ++q) {
        if (!g.act[q]) continue;
#pragma unroll
        for (int u = 0; u < EPT / R1; ++u)
#pragma unroll
          for (int r = 0; r < R1; ++r) {
            const int n = out_pos(q, u, r);
            cx<T> w = tw[n];
            w.y = -w.y;
            buf[f.vs.addr(g.vec[q], n)] = acc[q][u * R1 + r] + g.v[q][u * R1 + r] * w;
          }
      }
    }
  });
}

template <typename T, int M, bool BANDED = false>
__device__ __forceinline__ void col_conv(cx<T>* buf, const cx<T>* tw, const cx<T>* ghat, bool adjoint,
                                         int ncols = 2 * M, int kmin = 0) {
  using C = ConvCfg<T, M>;
  typename C::Cols cols;
  cols.nv = ncols;
  auto spec_col = [&](int c) {
    if constexpr (BANDED) {
      if (c < M) return 2 * c + 1;
      const int k = kmin + c - M;  // in (-M, M)
      return 2 * (k < 0 ? k + M : k);
    } else {
      return c;
    }
  };
  col_chains<T, M, C::EPT_C, C::NT>(buf, tw, ghat, adjoint, cols, spec_col);
  __syncthreads();  // the row pass that follows reads every column
}

// x -> G_D x (or G_D^H x) for x on the M x M block of the region at element
// offset src of the tile (0, or BOT with PP); returns the offset of the
// region holding the result.  Row passes are workgroup-wide (in place, or
// with PP alternating between the two regions); the column phase is
// wave-local, works in the region the rows end in, and ends with a workgroup
// barrier.
template <typename T, int M, bool PP>
__device__ __forceinline__ int conv_core(cx<T>* buf, const cx<T>* tw, const cx<T>* ghat, bool adjoint, int src) {
  using C = ConvCfg<T, M>;
  constexpr int P = C::P, BOT = C::BOT;
  const Fft<T, P, C::EPT_R, C::NT, typename C::Rows, 1> rows{buf, tw, typename C::Rows{}};
  if constexpr (PP) {
    const int r = rows.template run_pp<-1, M, P>(src, src == 0 ? BOT : 0);  // right halves are zero padding
    col_conv<T, M>(buf + r, tw, ghat, adjoint);
    return rows.template run_pp<+1, P, M>(r, r == 0 ? BOT : 0);            // only the left halves are kept
  } else {
    rows.template run<-1, M, P>(NoLoad(), src);
    col_conv<T, M>(buf + src, tw, ghat, adjoint);
    rows.template run<+1, P, M>(NoLoad(), src);
    return src;
  }
}

__device__ __forceinline__ int wrap_mode(int k, int M) { return ((k % M) + M) % M; }

// The 2M half-rows of the M x P tile as vectors of length M: vector v is the
// left (v even) or right (v odd) half of row v / 2.
template <int P>
struct HalfRows {
  static constexpr int NV = P;
  static constexpr bool WL = false;
  int nv = P;
  __device__ __forceinline__ int addr(int v, int k) const { return (v >> 1) * Tile<P>::LD + (v & 1) * (P / 2) + k; }
};

// First-pass load of x[k] w[k], w[k] = exp(-2 pi i k / P) (tw holds the P-point twiddles).
template <typename T>
struct TwistLoad {
  const cx<T>* tw;
  template <typename C>
  __device__ __forceinline__ C operator()(int, int k, C v) const { return v * tw[k]; }
};

template <typename T>
struct FwdArgs {
  const cx<T>* in;     // alpha [BP][K][K] (from_alpha) or pixel currents [BP][N]
  const cx<T>* einc;   // [Ni][N] incident fields, or null (taken as zero)
  const cx<T>* ghat;   // [P][P] spectrum / P^2
  const cx<T>* tw;     // [P] exp(-2 pi i k / P)
  cx<T>* J;            // [BP][N] synthesised currents (from_alpha), may be null
  cx<T>* E;            // [BP][N] output E_inc + G_D J + beta J
  int Ni, K;
  T beta;
};

// alpha -> J = F_T^*(alpha) (zero-filled inverse FFT), then
// E = E_inc + G_D J + beta J (Sec. 2.2, Eq. 6; Sec. 2.3, Eq. 9).
//
// From the coefficients the convolution uses that J is band-limited: with
// U[y][kx] the inverse column transforms of the K kept mode columns, the even
// frequencies of each zero-padded row's length-P transform are M U[y][k]
// (nonzero for the K kept k only) and the odd ones are FFT_M(J[y][.] w),
// w[x] = exp(-2 pi i x / P).  The tile holds the odd frequencies in columns
// 0..M-1 and the K even ones in columns M..M+K-1, so the column phase
// convolves M + K columns instead of 2M; the cropped inverse row transform is
// then IFFT_M(even) + conj(w) IFFT_M(odd) on the two halves of each row.
// With 2K <= M (grids up to 64), beta J joins in the row spectrum: J's row transform is M U on
// the kept columns, so beta U waits in the free columns M+K..M+2K-1 through
// the column phase and is added to the even half before its inverse, and E
// needs no second read of the stored J (equal to adding it up to FP32 or FP64
// rounding).  From given currents (the start value) the general convolution runs.
// PP: the plan of the row passes of the general convolution (see ConvCfg), a
// tuning choice with identical results; the band-limited path has one plan.
template <typename T, int M, bool FROM_ALPHA, bool PP>
__device__ __forceinline__ void fwd_conv_body(const FwdArgs<T>& a, int bp, unsigned char* smem_raw) {
  using C = ConvCfg<T, M>;
  constexpr int P = C::P;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + (PP ? 2 : 1) * C::M * C::TileL::LD;
  const int p = bp % a.Ni;
  const int tid = threadIdx.x;
  const size_t off = size_t(bp) * C::N;
  // epilogue loads (issued early: nothing else on the CU hides their latency)
  auto load_einc = [&](cx<T>(&ei)[C::PPT]) {
    if (a.einc) {
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) ei[q] = a.einc[size_t(p) * C::N + tid + q * C::NT];
    } else {
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) ei[q] = cx<T>{T(0), T(0)};
    }
  };
  if constexpr (FROM_ALPHA) {
    // the coefficients (K^2 <= N) are loaded with the twiddles in one round trip
    const int K = a.K, KK = K * K, kmin = -(K / 2);
    const cx<T>* al = a.in + size_t(bp) * KK;
    cx<T> av[C::PPT];
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) av[q] = al[min(tid + q * C::NT, KK - 1)];
    for (int k = tid; k < P; k += C::NT) tw[k] = a.tw[k];
    // the M x M block starts at zero: the mode passes transform only the K kept columns
    for (int e = tid; e < C::N; e += C::NT) buf[C::TileL::at(e / M, e % M)] = cx<T>{T(0), T(0)};
    __syncthreads();
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      const int e = tid + q * C::NT;
      if (e < KK) buf[C::TileL::at(wrap_mode(kmin + e / K, M), wrap_mode(kmin + e % K, M))] = av[q];
    }
    __syncthreads();
    // U: inverse transforms along y of the K kept mode columns
    typename C::ModeCols mc;
    mc.nv = K;
    mc.kmin = kmin;
    Fft<T, M, C::EPT_M, C::NT, typename C::ModeCols, 2>{buf, tw, mc}.template run<+1>();
    // even frequencies M U[y][k] of the kept k, compact in columns M..M+K-1 (and
    // beta U in columns M+K..M+2K-1 when they fit)
    const bool bj = M <= 64 && 2 * K <= M;  // at 96 the second epilogue would add spills
    for (int e = tid; e < M * K; e += C::NT) {
      const int y = e / K, j = e % K;
      const cx<T> u = buf[C::TileL::at(y, wrap_mode(kmin + j, M))];
      buf[C::TileL::at(y, M + j)] = T(M) * u;
      if (bj) buf[C::TileL::at(y, M + K + j)] = a.beta * u;
    }
    // (the next pass stores to columns 0..M-1 only after its first barrier)
    // J: inverse transforms along x of all M rows
    Fft<T, M, C::EPT_M, C::NT, typename C::RowsM, 2> rowsm{buf, tw, typename C::RowsM{}};
    rowsm.template run<+1>();
    // J goes to its output now and is read back by the same threads in the
    // epilogue (still in L2), which keeps it out of the registers the column
    // phase needs; J is required here
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      const int n = tid + q * C::NT;
      a.J[off + n] = buf[C::TileL::at(n / M, n % M)];
    }
    // odd frequencies FFT_M(J w) of each row, in place in columns 0..M-1
    rowsm.template run<-1>(TwistLoad<T>{tw});
    col_conv<T, M, true>(buf, tw, a.ghat, false, M + K, kmin);
    // even part back to natural order (zero where no mode is kept; plus beta U) in columns M..P-1
    cx<T> ev[C::PPT];
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      const int e = tid + q * C::NT;
      const int y = e / M, k = e % M, j = wrap_mode(k - kmin, M);
      ev[q] = cx<T>{T(0), T(0)};
      if (j < K) {
        ev[q] = buf[C::TileL::at(y, M + j)];
        if (bj) ev[q] = ev[q] + buf[C::TileL::at(y, M + K + j)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      const int e = tid + q * C::NT;
      buf[C::TileL::at(e / M, M + e % M)] = ev[q];
    }
    __syncthreads();
    // inverse transforms of both halves of every row
    Fft<T, M, C::EPT_M, C::NT, HalfRows<P>, 2>{buf, tw, HalfRows<P>{}}.template run<+1>();
    cx<T> ei[C::PPT];
    load_einc(ei);
    if (bj) {
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) {
        const int n = tid + q * C::NT, y = n / M, x = n % M;
        cx<T> w = tw[x];
        w.y = -w.y;
        a.E[off + n] = buf[C::TileL::at(y, M + x)] + buf[C::TileL::at(y, x)] * w + ei[q];
      }
    } else {
      cx<T> jr[C::PPT];
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) jr[q] = a.J[off + tid + q * C::NT];
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) {
        const int n = tid + q * C::NT, y = n / M, x = n % M;
        cx<T> w = tw[x];
        w.y = -w.y;
        a.E[off + n] = buf[C::TileL::at(y, M + x)] + buf[C::TileL::at(y, x)] * w + a.beta * jr[q] + ei[q];
      }
    }
  } else {
    cx<T> jr[C::PPT];
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) jr[q] = a.in[off + tid + q * C::NT];
    for (int k = tid; k < P; k += C::NT) tw[k] = a.tw[k];
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      const int n = tid + q * C::NT;
      buf[C::TileL::at(n / M, n % M)] = jr[q];
    }
    __syncthreads();
    const int res = conv_core<T, M, PP>(buf, tw, a.ghat, false, 0);
    cx<T> ei[C::PPT];
    load_einc(ei);
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      const int n = tid + q * C::NT;
      a.E[off + n] = buf[res + C::TileL::at(n / M, n % M)] + a.beta * jr[q] + ei[q];
    }
  }
}

template <typename T, int M, bool FROM_ALPHA, bool PP>
__global__ __launch_bounds__((ConvCfg<T, M>::NT), (ConvCfg<T, M>::wpe(PP))) void k_fwd_conv(FwdArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fwd_conv_body<T, M, FROM_ALPHA, PP>(a, blockIdx.x, smem_raw);
}

// One launch over several argument sets (handles of one shape class).
template <typename T, int M, bool FROM_ALPHA, bool PP>
__global__ __launch_bounds__((ConvCfg<T, M>::NT), (ConvCfg<T, M>::wpe(PP))) void k_fwd_conv_group(const FwdArgs<T>* __restrict__ a,
                                                                         const int* __restrict__ start, int n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = group_of(start, n, blockIdx.x);
  fwd_conv_body<T, M, FROM_ALPHA, PP>(a[g], blockIdx.x - start[g], smem_raw);
}

// ---- the band-limited forward on a compact tile
//
// From coefficients the tile needs only the M odd-frequency columns and the K
// kept even ones, so a tile of M rows x (M + KC) columns (KC >= K) serves, and
// column chains of 8 elements per thread keep the registers low: at M = 64 in
// FP32 (KC = 32: 50 KB) three 512-thread workgroups share a CU instead of two.
// The odd columns take one chain per 8 lanes on all wavefronts, the K even
// columns a second round on the first wavefronts.  The cropped inverse row
// transform runs on the M x M block twice: the odd part (times conj(w)) into
// registers, then the even part placed back in natural order.  Same
// arithmetic as fwd_conv_body up to the radices of the column chains.
template <typename T, int M>
struct CompactCfg {
  static constexpr int KC = M / 2;            // largest K on the compact tile
  static constexpr int PC = M + KC;           // row: M odd-frequency (pixel) columns, then KC even ones
  using TileC = Tile<PC>;                     // row stride PC + 1 (odd)
  static constexpr int NT = ConvCfg<T, M>::NT;
  static constexpr int N = M * M, PPT = N / NT;
  static constexpr int EPT = 8;               // basis transforms and column chains
  // + the P twiddles (forward), and the half-shift values over two periods (adjoint)
  static constexpr size_t LDS = sizeof(cx<T>) * (size_t(M) * TileC::LD + 2 * M);
  static constexpr size_t LDS_ADJ = LDS + sizeof(cx<T>) * 2 * M;
  static constexpr int WPE = int((160 * 1024) / LDS_ADJ) * (NT / 64) / 4 > 8 ? 8 : int((160 * 1024) / LDS_ADJ) * (NT / 64) / 4;
  using RowsM = Vecs<PC, M, true>;
  using ModeCols = Vecs<PC, M, false, true>;
};

// Wave-local columns c0 .. c0 + nv - 1 of a Tile<TP> (at most NV of them).
template <int TP, int NV_>
struct OffCols {
  static constexpr int NV = NV_;
  static constexpr bool WL = true;
  int nv = NV_;
  int c0 = 0;
  __device__ __forceinline__ int addr(int v, int k) const { return Tile<TP>::at(k, c0 + v); }
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Row products on the matrix cores for the compact tile (64 x 64 FP32).  The
// complex product Y = X C is the real one
//   [Re Y, Im Y] = [Re X, Im X] [[Re C, Im C], [-Im C, Re C]]
// on v_mfma_f32_16x16x4f32, two complex input columns per instruction: lane
// l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and register e returns
// D[e + 4 (l / 16)][l % 16].  So lane l works on row i = l % 16 of A, on part
// l / 16 % 2 (0 Re, 1 Im) of input column (l / 16) / 2 of a step, and on
// output column (l % 16) / 2, part l % 2; B takes component sel = (l / 16 %
// 2) xor (l % 2) of C, negated for A's imaginary part against a real output.
// Every output sums over the input columns in one fixed order.
//
// The coefficients are the half-shift values hs[m] = 2 / (1 - exp(-i pi (2m
// + 1) / M)), stored after the P twiddles (layout at kept_rows_hs): with
// w[x] = exp(-2 pi i x / P),
//   sum_x w[x] exp(2 pi i (k - c) x / M) = hs[(c - k) mod M]
// (a geometric sum of ratio exp(-i pi (2 (c - k) + 1) / M), whose M-th power
// is -1), i.e. the length-M transform of w times one mode.
struct RowProdLane {
  int i, kq, pa, sel;
  float sg;
  __device__ __forceinline__ RowProdLane() {
    const int l = threadIdx.x & 63;
    i = l & 15;
    kq = l >> 4;
    pa = kq & 1;
    sel = pa ^ (i & 1);
    sg = (pa == 1 && (i & 1) == 0) ? -1.f : 1.f;
  }
};

// Y[r][j] = s sum_{c < M} X[r][c] conj(hs[c - k_j]) for r < M and j < K <= 16
// (k_j = kmin + j), X the first M columns of the tile; wave w of eight takes
// rows 16 (w % 4) .. + 15 and outputs 8 (w / 4) .. + 7.  This lane's results:
// acc[e] is part `part` of Y[row + e][j] (valid for j < K).  The half-shift
// values are stored over two periods from -M/2 (tw[P + p] = hs[(p - M/2) mod
// M], p < 2M; index c - k_j + M/2 lies in [M/2 - K/2, 3M/2 + K/2) for c < M),
// so that a lane's coefficients of successive steps sit at constant offsets;
// the even and the odd steps accumulate separately and are added at the end.
struct KeptOut {
  f32x4 acc;
  int row, j, part;
};
template <int M, int LD>
__device__ __forceinline__ KeptOut kept_rows_hs(const cx<float>* buf, const cx<float>* tw, int K, int kmin,
                                                float scale) {
  const RowProdLane ln;
  const int w = threadIdx.x >> 6;
  KeptOut o;
  o.row = 16 * (w & 3) + 4 * ln.kq;
  o.j = 8 * (w >> 2) + (ln.i >> 1);
  o.part = ln.i & 1;
  o.acc = f32x4{0.f, 0.f, 0.f, 0.f};
  if (8 * (w >> 2) >= K) return o;  // no output column of this wave
  const int jc = o.j < K ? o.j : K - 1;
  // the role's sign, conj on the imaginary component, and the scale
  const float f = o.j < K ? (ln.sel ? -ln.sg : ln.sg) * scale : 0.f;
  const float* xr = reinterpret_cast<const float*>(buf + (16 * (w & 3) + ln.i) * LD) + 2 * (ln.kq >> 1) + ln.pa;
  // step s reads table entry 2 s + (kq / 2) - k_j + M/2
  const float* hr = reinterpret_cast<const float*>(tw + 2 * M + (ln.kq >> 1) - (kmin + jc) + M / 2) + ln.sel;
  f32x4 a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < M / 2; s += 2) {
    o.acc = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[4 * s], f * hr[4 * s], o.acc, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[4 * s + 4], f * hr[4 * s + 4], a1, 0, 0, 0);
  }
  o.acc = o.acc + a1;
  return o;
}

__device__ __forceinline__ void set_part(cx<float>& z, int part, float v) {
  reinterpret_cast<float*>(&z)[part] = v;
}

// BJ (K <= 16): beta J joins in the row spectrum instead of the pixel domain.
// J's row transform is M U on the kept columns, so beta U waits in the spare
// columns M + K .. M + 2K - 1 through the column phase and is added to the
// convolved even columns before their inverse row transform; E then needs no
// second read of the J this kernel stored (the result differs from adding the
// stored J by FP32 rounding only).
template <typename T, int M, bool BJ>
__device__ __forceinline__ void fwd_conv_compact_body(const FwdArgs<T>& a, int bp, unsigned char* smem_raw) {
  using C = CompactCfg<T, M>;
  using TC = typename C::TileC;
  constexpr int NT = C::NT, PPT = C::PPT;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + M * TC::LD;
  const int p = bp % a.Ni;
  const int tid = threadIdx.x;
  const size_t off = size_t(bp) * C::N;
  const int K = a.K, KK = K * K, kmin = -(K / 2);
  const cx<T>* al = a.in + size_t(bp) * KK;
  cx<T> av[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) av[q] = al[min(tid + q * NT, KK - 1)];
  for (int k = tid; k < 2 * M; k += NT) tw[k] = a.tw[k];
  for (int e = tid; e < C::N; e += NT) buf[TC::at(e / M, e % M)] = cx<T>{T(0), T(0)};
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int e = tid + q * NT;
    if (e < KK) buf[TC::at(wrap_mode(kmin + e / K, M), wrap_mode(kmin + e % K, M))] = av[q];
  }
  __syncthreads();
  // U: inverse transforms along y of the K kept mode columns
  typename C::ModeCols mc;
  mc.nv = K;
  mc.kmin = kmin;
  Fft<T, M, C::EPT, NT, typename C::ModeCols, 2>{buf, tw, mc}.template run<+1>();
  // even frequencies M U[y][k] of the kept k, compact in columns M..M+K-1
  // (BJ: and beta U in columns M+K..M+2K-1)
  for (int e = tid; e < M * K; e += NT) {
    const int y = e / K, j = e % K;
    const cx<T> u = buf[TC::at(y, wrap_mode(kmin + j, M))];
    buf[TC::at(y, M + j)] = T(M) * u;
    if constexpr (BJ) buf[TC::at(y, M + K + j)] = a.beta * u;
  }
  // J: inverse transforms along x of all M rows (the first pass stores only after its barrier)
  const Fft<T, M, C::EPT, NT, typename C::RowsM, 2> rowsm{buf, tw, typename C::RowsM{}};
  rowsm.template run<+1>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n = tid + q * NT;
    a.J[off + n] = buf[TC::at(n / M, n % M)];
  }
  // odd frequencies FFT_M(J w) of each row, in place
  rowsm.template run<-1>(TwistLoad<T>{tw});
  // the column phase: the M odd columns (spectrum column 2c + 1), then the K even ones
  {
    OffCols<C::PC, M> odd;
    col_chains<T, M, C::EPT, NT>(buf, tw, a.ghat, false, odd, [](int c) { return 2 * c + 1; });
    OffCols<C::PC, C::KC> even;
    even.nv = K;
    even.c0 = M;
    col_chains<T, M, C::EPT, NT>(buf, tw, a.ghat, false, even, [&](int j) { return 2 * wrap_mode(kmin + j, M); });
  }
  __syncthreads();
  // the odd part: conj(w) IFFT_M of each row, kept per pixel
  rowsm.template run<+1>();
  cx<T> eo[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n = tid + q * NT, x = n % M;
    cx<T> w = tw[x];
    w.y = -w.y;
    eo[q] = buf[TC::at(n / M, x)] * w;
  }
  __syncthreads();
  // the even part in natural order (zero where no mode is kept; BJ: plus beta U), then its inverse
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n = tid + q * NT, y = n / M, j = wrap_mode(n % M - kmin, M);
    cx<T> z{T(0), T(0)};
    if (j < K) {
      z = buf[TC::at(y, M + j)];
      if constexpr (BJ) z = z + buf[TC::at(y, M + K + j)];
    }
    buf[TC::at(y, n % M)] = z;
  }
  __syncthreads();
  rowsm.template run<+1>();
  cx<T> ei[PPT];
  if (a.einc) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) ei[q] = a.einc[size_t(p) * C::N + tid + q * NT];
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) ei[q] = cx<T>{T(0), T(0)};
  }
  if constexpr (BJ) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int n = tid + q * NT;
      a.E[off + n] = buf[TC::at(n / M, n % M)] + eo[q] + ei[q];
    }
  } else {
    cx<T> jr[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) jr[q] = a.J[off + tid + q * NT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int n = tid + q * NT;
      a.E[off + n] = buf[TC::at(n / M, n % M)] + eo[q] + a.beta * jr[q] + ei[q];
    }
  }
}

template <typename T, int M, bool BJ>
__global__ __launch_bounds__((CompactCfg<T, M>::NT), (CompactCfg<T, M>::WPE)) void k_fwd_conv_c(FwdArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fwd_conv_compact_body<T, M, BJ>(a, blockIdx.x, smem_raw);
}

template <typename T, int M, bool BJ>
__global__ __launch_bounds__((CompactCfg<T, M>::NT), (CompactCfg<T, M>::WPE)) void k_fwd_conv_c_group(
    const FwdArgs<T>* __restrict__ a, const int* __restrict__ start, int n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = group_of(start, n, blockIdx.x);
  fwd_conv_compact_body<T, M, BJ>(a[g], blockIdx.x - start[g], smem_raw);
}

template <typename T>
struct AdjArgs {
  const cx<T>* J;      // [BP][N] currents, or null (alpha = 0)
  const cx<T>* E;      // [BP][N], or [Ni][N] if e_shared
  int e_shared;
  const cx<T>* h;      // [BP][N] G_S^H (data residual or measured field)
  const cx<T>* R;      // [B][N]
  const cx<T>* Rs;     // [B][N] contrast of the state residual, or null (R): R_c with the loss on the CCO image
  const T* den;        // [B][N]  sum_p |E_p|^2
  const cx<T>* gR;     // [B][N] dL/dR from the regularisers, or null
  const double* Ss;    // ||E_inc||^2 (scalar)
  const double* Sd;    // [B] ||E_sca||^2
  double hsign;        // sign applied to h
  const cx<T>* ghat;
  const cx<T>* tw;
  cx<T>* galpha;       // [BP][K][K] gradient output, or null
  cx<T>* alpha;        // Adam: parameters updated in place (null: no update)
  T* m;
  T* v;
  const int* frozen;   // [B] nonzero: skip the update, or null
  T gr_w;              // weight of the regulariser part (1; 1 / ||E_inc,f||^2 when den sums frequencies)
  const double* adam_c;  // [B][2] lr / (1 - b1^t), 1 / (1 - b2^t) of this step (with alpha)
  double b1, b2, eps;
  int Ni, K;
  T beta;
};

// Adjoint of the loss (chain rule through Eqs. 6-7, 9, 15-16):
//   g_s = 2 s / ||E_inc||^2,  s = R E - beta J
//   g_E = conj(R) g_s + (beta conj(g_R) J - 2 Re(conj(g_R) R) E) / den
//   g_J = -beta g_s + beta g_R E / den + beta g_E + G_D^H g_E + 2 G_S^H d / ||E_sca||^2
//   g_alpha = B^H g_J  (unnormalised forward DFT on the kept modes)
// The state loss's own derivative in R vanishes because R is its per-pixel
// least-squares minimiser, so only the regulariser part g_R reaches R.  With
// the loss on the CCO image the residual takes R_c (Rs) in s and in g_E's
// first term, and g_R carries the state term through the CCO as well.
// The adjoint's per-pixel part: g_E and g_J of the pixels n = tid + q NT (q <
// PPT) handed to emit(q, n, g_E, g_J).  The loads are issued in batches of QB
// pixels per thread, all loads of a batch before their use; optional inputs
// are uniform branches around whole groups of loads.  Batches bound the
// registers live next to g_J, which the callers keep through the convolution.
template <typename T, int M, int NT, class Emit>
__device__ __forceinline__ void adj_pixels(const AdjArgs<T>& a, int bp, const Emit& emit) {
  constexpr int N = M * M, PPT = N / NT;
  const int b = bp / a.Ni, p = bp % a.Ni;
  const int tid = threadIdx.x;
  const size_t off = size_t(bp) * N;
  const size_t eoff = size_t(a.e_shared ? p : bp) * N;
  const size_t boff = size_t(b) * N;
  const T ws = T(2) / T(a.Ss[0]);
  const T wd = T(2 * a.hsign) / T(a.Sd[b]);
  const T beta = a.beta;
  constexpr int QB = PPT <= 4 ? PPT : (PPT % 4 == 0 ? 4 : (PPT % 3 == 0 ? 3 : (PPT % 2 == 0 ? 2 : 1)));
  static_assert(PPT % QB == 0, "whole batches");
  const bool has_j = a.J != nullptr, has_gr = a.gR != nullptr, has_rs = a.Rs != nullptr;
#pragma unroll
  for (int q0 = 0; q0 < PPT; q0 += QB) {
    cx<T> Jv[QB], Ev[QB], Rv[QB], Hv[QB], Gv[QB], Sv[QB];
    T Dv[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int n = tid + (q0 + q) * NT;
      Ev[q] = a.E[eoff + n];
      Rv[q] = a.R[boff + n];
      Hv[q] = a.h[off + n];
    }
    if (has_j) {
#pragma unroll
      for (int q = 0; q < QB; ++q) Jv[q] = a.J[off + tid + (q0 + q) * NT];
    } else {
#pragma unroll
      for (int q = 0; q < QB; ++q) Jv[q] = cx<T>{T(0), T(0)};
    }
    if (has_gr) {
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        Gv[q] = a.gR[boff + tid + (q0 + q) * NT];
        Dv[q] = a.den[boff + tid + (q0 + q) * NT];
      }
    }
    if (has_rs) {
#pragma unroll
      for (int q = 0; q < QB; ++q) Sv[q] = a.Rs[boff + tid + (q0 + q) * NT];
    } else {
#pragma unroll
      for (int q = 0; q < QB; ++q) Sv[q] = Rv[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int n = tid + (q0 + q) * NT;
      const cx<T> J = Jv[q], E = Ev[q], R = Rv[q], Rs = Sv[q];
      const cx<T> s = Rs * E - beta * J;
      const cx<T> gs = ws * s;
      cx<T> gE = cmul_conj_a(Rs, gs);
      cx<T> gJ = (-beta) * gs + wd * Hv[q];
      if (has_gr) {
        const cx<T> g = Gv[q];
        const T inv = a.gr_w / Dv[q];
        const T re = g.x * R.x + g.y * R.y;  // Re(conj(g) R)
        gE = gE + inv * (beta * cmul_conj_a(g, J) - (T(2) * re) * E);
        gJ = gJ + (beta * inv) * (g * E);
      }
      gJ = gJ + beta * gE;
      emit(q0 + q, n, gE, gJ);
    }
  }
}

// g_alpha of the K x K kept modes read(iy, ix) of the analysed tile, and the
// Adam update of alpha (bias corrections of this step from adam_c).
template <typename T, int M, int NT, class Read>
__device__ __forceinline__ void adj_modes(const AdjArgs<T>& a, int bp, const Read& read) {
  const int b = bp / a.Ni, tid = threadIdx.x;
  const int K = a.K, kmin = -(K / 2);
  const bool upd = a.alpha && !(a.frozen && a.frozen[b]);
  T lr1 = T(0), ic2 = T(0);
  if (upd) {
    lr1 = T(a.adam_c[2 * b]);
    ic2 = T(a.adam_c[2 * b + 1]);
  }
  for (int e = tid; e < K * K; e += NT) {
    const int iy = wrap_mode(kmin + e / K, M), ix = wrap_mode(kmin + e % K, M);
    const cx<T> g = read(iy, ix);
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

template <typename T, int M, bool PP>
__device__ __forceinline__ void adj_conv_body(const AdjArgs<T>& a, int bp, unsigned char* smem_raw) {
  using C = ConvCfg<T, M>;
  constexpr int GJL = C::gj_lds(PP);
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + (PP ? 2 : 1) * C::M * C::TileL::LD;
  const int tid = threadIdx.x;
  for (int k = tid; k < C::P; k += C::NT) tw[k] = a.tw[k];
  cx<T> gj[C::PPT];
  cx<T>* gjs = tw + C::P;  // [GJ_LDS][NT], each thread's own entries
  adj_pixels<T, M, C::NT>(a, bp, [&](int q, int n, const cx<T>& gE, const cx<T>& gJ) {
    buf[C::TileL::at(n / M, n % M)] = gE;
    if (q < GJL)
      gjs[q * C::NT + tid] = gJ;
    else
      gj[q] = gJ;
  });
  __syncthreads();
  const int r = conv_core<T, M, PP>(buf, tw, a.ghat, true, 0);  // offset of the result in the tile
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) {
    const int n = tid + q * C::NT;
    cx<T>& x = buf[r + C::TileL::at(n / M, n % M)];
    x = x + (q < GJL ? gjs[q * C::NT + tid] : gj[q]);
  }
  __syncthreads();
  const int K = a.K, kmin = -(K / 2);
  Fft<T, M, C::EPT_M, C::NT, typename C::RowsM, 2>{buf, tw, typename C::RowsM{}}.template run<-1>(NoLoad(), r);
  typename C::ModeCols mc;
  mc.nv = K;
  mc.kmin = kmin;
  Fft<T, M, C::EPT_M, C::NT, typename C::ModeCols, 2>{buf, tw, mc}.template run<-1>(NoLoad(), r);
  adj_modes<T, M, C::NT>(a, bp, [&](int iy, int ix) { return buf[r + C::TileL::at(iy, ix)]; });
}

// First-pass load of the kept mode column j (row k) plus s times column OFF + j
// of the same row of a Tile<TP> (the compact even frequencies) and, with
// GJ, plus column OFF + K + j (the kept columns of the row transform of g_J).
template <typename T, int TP, int OFF, bool GJ>
struct EvenJoinLoad {
  const cx<T>* buf;
  T s;
  int K;
  template <typename Cx>
  __device__ __forceinline__ Cx operator()(int j, int k, Cx x) const {
    x = x + s * buf[Tile<TP>::at(k, OFF + j)];
    if constexpr (GJ) x = x + buf[Tile<TP>::at(k, OFF + K + j)];
    return x;
  }
};

// The adjoint on the compact tile (64 x 64 FP32, K <= 32; as the compact
// forward).  Only the K x K kept modes of B^H (G_D^H g_E + g_J) are wanted:
// with the padded row transform's even and odd frequencies (Z_even =
// FFT_M(g_E), Z_odd = FFT_M(w g_E) per row, w[x] = exp(-2 pi i x / P)), the
// column phase with conj(ghat) gives W_even, W_odd and
//   G_D^H g_E = IFFT_M(W_even) + conj(w) IFFT_M(W_odd)   (per row);
// B^H takes the first term to M times the kept columns of W_even under the
// column transform, so only the K kept even columns are convolved:
//   g_alpha = colFFT_kept(M W_even + rowFFT(conj(w) IFFT_M(W_odd)) + rowFFT(g_J)).
// g_E waits in registers between its row transforms.  GJ (K <= 16): the kept
// columns of rowFFT(g_J) are formed first and wait in the compact tile's
// spare columns M + K.., so no g_J is held through the convolution (the
// registers it would take push the column phase past the 80 that three
// workgroups per CU leave), and the odd part's two row transforms are one
// product on the matrix cores with the half-shift values (only its K kept
// columns are needed); otherwise g_J waits in registers and joins in the
// pixel domain.
template <typename T, int M, bool GJ>
__device__ __forceinline__ void adj_conv_compact_body(const AdjArgs<T>& a, int bp, unsigned char* smem_raw) {
  using C = CompactCfg<T, M>;
  using TC = typename C::TileC;
  constexpr int NT = C::NT, PPT = C::PPT;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + M * TC::LD;
  const int tid = threadIdx.x;
  for (int k = tid; k < 4 * M; k += NT) tw[k] = a.tw[k];
  const int K = a.K, kmin = -(K / 2);
  const Fft<T, M, C::EPT, NT, typename C::RowsM, 2> rowsm{buf, tw, typename C::RowsM{}};
  cx<T> ge[PPT], gj[GJ ? 1 : PPT];
  if constexpr (GJ) {
    adj_pixels<T, M, NT>(a, bp, [&](int q, int n, const cx<T>& gE, const cx<T>& gJ) {
      buf[TC::at(n / M, n % M)] = gJ;
      ge[q] = gE;
    });
    __syncthreads();
    rowsm.template run<-1>();
    for (int e = tid; e < M * K; e += NT) {
      const int y = e / K, j = e % K;
      buf[TC::at(y, M + K + j)] = buf[TC::at(y, wrap_mode(kmin + j, M))];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int n = tid + q * NT;
      buf[TC::at(n / M, n % M)] = ge[q];
    }
  } else {
    adj_pixels<T, M, NT>(a, bp, [&](int q, int n, const cx<T>& gE, const cx<T>& gJ) {
      buf[TC::at(n / M, n % M)] = gE;
      ge[q] = gE;
      gj[q] = gJ;
    });
  }
  __syncthreads();
  // even frequencies FFT_M(g_E) of each row; the K kept ones compact in columns M..M+K-1
  rowsm.template run<-1>();
  for (int e = tid; e < M * K; e += NT) {
    const int y = e / K, j = e % K;
    buf[TC::at(y, M + j)] = buf[TC::at(y, wrap_mode(kmin + j, M))];
  }
  __syncthreads();
  // odd frequencies FFT_M(w g_E) of each row, in place
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n = tid + q * NT;
    buf[TC::at(n / M, n % M)] = ge[q];
  }
  __syncthreads();
  rowsm.template run<-1>(TwistLoad<T>{tw});
  // the column phase with conj(ghat): the M odd columns, then the K kept even ones
  {
    OffCols<C::PC, M> odd;
    col_chains<T, M, C::EPT, NT>(buf, tw, a.ghat, true, odd, [](int c) { return 2 * c + 1; });
    OffCols<C::PC, C::KC> even;
    even.nv = K;
    even.c0 = M;
    col_chains<T, M, C::EPT, NT>(buf, tw, a.ghat, true, even, [&](int j) { return 2 * wrap_mode(kmin + j, M); });
  }
  __syncthreads();
  if constexpr (GJ) {
    // the odd part: the kept columns of FFT_M(conj(w) IFFT_M(W_odd)) = sum_c W_odd[c] conj(hs[c - k_j]),
    // to their natural columns once every wave has read W_odd (matrix cores)
    const KeptOut o = kept_rows_hs<M, TC::LD>(buf, tw, K, kmin, T(1));
    __syncthreads();
    if (o.j < K)
#pragma unroll
      for (int e = 0; e < 4; ++e) set_part(buf[TC::at(o.row + e, wrap_mode(kmin + o.j, M))], o.part, o.acc[e]);
  } else {
    // the odd part back to pixels, conj(w) IFFT_M, plus g_J, then the row transform
    rowsm.template run<+1>();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int n = tid + q * NT, x = n % M;
      cx<T> w = tw[x];
      w.y = -w.y;
      cx<T>& d = buf[TC::at(n / M, x)];
      d = d * w + gj[q];
    }
    __syncthreads();
    rowsm.template run<-1>();
  }
  __syncthreads();
  // column transforms of the kept modes, M W_even (and rowFFT(g_J)) joining in their first pass
  typename C::ModeCols mc;
  mc.nv = K;
  mc.kmin = kmin;
  Fft<T, M, C::EPT, NT, typename C::ModeCols, 2>{buf, tw, mc}.template run<-1>(
      EvenJoinLoad<T, C::PC, M, GJ>{buf, T(M), K});
  adj_modes<T, M, NT>(a, bp, [&](int iy, int ix) { return buf[TC::at(iy, ix)]; });
}

template <typename T, int M, bool GJ>
__global__ __launch_bounds__((CompactCfg<T, M>::NT), (CompactCfg<T, M>::WPE)) void k_adj_conv_c(AdjArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  adj_conv_compact_body<T, M, GJ>(a, xcd_remap(blockIdx.x, gridDim.x), smem_raw);
}

template <typename T, int M, bool GJ>
__global__ __launch_bounds__((CompactCfg<T, M>::NT), (CompactCfg<T, M>::WPE)) void k_adj_conv_c_group(
    const AdjArgs<T>* __restrict__ a, const int* __restrict__ start, int n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int bx = xcd_remap(blockIdx.x, gridDim.x);
  const int g = group_of(start, n, bx);
  adj_conv_compact_body<T, M, GJ>(a[g], bx - start[g], smem_raw);
}

template <typename T, int M, bool PP>
__global__ __launch_bounds__((ConvCfg<T, M>::NT), (ConvCfg<T, M>::wpe(PP))) void k_adj_conv(AdjArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the N_i workgroups of an instance read its per-pixel R, den and g_R: one XCD serves them
  adj_conv_body<T, M, PP>(a, xcd_remap(blockIdx.x, gridDim.x), smem_raw);
}

template <typename T, int M, bool PP>
__global__ __launch_bounds__((ConvCfg<T, M>::NT), (ConvCfg<T, M>::wpe(PP))) void k_adj_conv_group(
    const AdjArgs<T>* __restrict__ a, const int* __restrict__ start, int n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int bx = xcd_remap(blockIdx.x, gridDim.x);
  const int g = group_of(start, n, bx);
  adj_conv_body<T, M, PP>(a[g], bx - start[g], smem_raw);
}

// alpha = F_T(J) on the kept modes (Sec. 2.3, Eq. 9): forward DFT of one
// set of pixel currents divided by M^2 (grid: one workgroup per current).
template <typename T, int M>
__global__ __launch_bounds__((ConvCfg<T, M>::NT), (ConvCfg<T, M>::WPE)) void k_analyze(const cx<T>* J, const cx<T>* twg, cx<T>* alpha,
                                                                  int K) {
  using C = ConvCfg<T, M>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + C::M * C::TileL::LD;
  const size_t v = blockIdx.x;
  const int tid = threadIdx.x;
  cx<T> jv[C::PPT];
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) jv[q] = J[v * C::N + tid + q * C::NT];
  for (int k = tid; k < C::P; k += C::NT) tw[k] = twg[k];
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) {
    const int n = tid + q * C::NT;
    buf[C::TileL::at(n / M, n % M)] = jv[q];
  }
  __syncthreads();
  const int kmin = -(K / 2);
  Fft<T, M, C::EPT_M, C::NT, typename C::RowsM, 2>{buf, tw, typename C::RowsM{}}.template run<-1>();
  typename C::ModeCols mc;
  mc.nv = K;
  mc.kmin = kmin;
  Fft<T, M, C::EPT_M, C::NT, typename C::ModeCols, 2>{buf, tw, mc}.template run<-1>();
  const T s = T(1) / T(C::N);
  for (int e = tid; e < K * K; e += C::NT) {
    const cx<T> g = buf[C::TileL::at(wrap_mode(kmin + e / K, M), wrap_mode(kmin + e % K, M))];
    alpha[v * K * K + e] = cx<T>{s * g.x, s * g.y};
  }
}

}  // namespace pdfk
