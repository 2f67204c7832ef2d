// Batched complex FFTs on data resident in LDS, for one workgroup.
//
// Radix-R Stockham autosort passes: each thread holds EPT elements of one
// vector in registers, does EPT/R radix-R butterflies per pass with the
// in-register FFTs below, and exchanges through LDS between passes (load all,
// barrier, store all, barrier), so the transform is in place and needs no
// bit reversal.  Vectors are rows or columns of a 2-D tile: element k of
// vector v sits at buf[v * vstride + k * estride].  Threads are assigned
// vector-fastest, so neighbouring lanes touch neighbouring rows / columns.
//
// Forward transforms use exp(-2 pi i jk/L) (DIR = -1), inverse ones
// exp(+2 pi i jk/L) (DIR = +1); neither is normalised.
#pragma once

#include "cplx.h"

namespace pdfk {

// cos(2 pi k / 16); sin(2 pi k / 16) = cos(2 pi (k - 4) / 16).
__host__ __device__ constexpr double cos16(int k) {
  switch (k & 15) {
    case 0: return 1.0;
    case 1: return 0.92387953251128675613;
    case 2: return 0.70710678118654752440;
    case 3: return 0.38268343236508977173;
    case 4: return 0.0;
    case 5: return -0.38268343236508977173;
    case 6: return -0.70710678118654752440;
    case 7: return -0.92387953251128675613;
    case 8: return -1.0;
    case 9: return -0.92387953251128675613;
    case 10: return -0.70710678118654752440;
    case 11: return -0.38268343236508977173;
    case 12: return 0.0;
    case 13: return 0.38268343236508977173;
    case 14: return 0.70710678118654752440;
    default: return 0.92387953251128675613;
  }
}

template <int R>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register FFT of R points (R = 1, 2, 4, 8, 16), natural order in and out.
template <typename T, int R, int DIR>
__device__ __forceinline__ void fft_reg(cx<T>* v) {
  if constexpr (R > 1) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = bitrev<R>(i);
      if (j > i) {
        cx<T> t = v[i];
        v[i] = v[j];
        v[j] = t;
      }
    }
#pragma unroll
    for (int s = 1; s < R; s <<= 1) {
#pragma unroll
      for (int k = 0; k < R; k += 2 * s) {
#pragma unroll
        for (int j = 0; j < s; ++j) {
          const int e = j * (16 / (2 * s));  // twiddle exp(DIR 2 pi i j / 2s) in 16ths
          const cx<T> w = {T(cos16(e)), T(DIR * cos16(e - 4))};
          cx<T> a = v[k + j];
          cx<T> b = (j == 0) ? v[k + j + s] : v[k + j + s] * w;
          v[k + j] = a + b;
          v[k + j + s] = a - b;
        }
      }
    }
  }
}

struct NoLoad {
  template <typename C>
  __device__ __forceinline__ C operator()(int, int, C v) const { return v; }
};
struct KeepAll {
  __device__ __forceinline__ bool operator()(int, int) const { return true; }
};

// One workgroup transforms nvec vectors of length L.  NT = blockDim.x,
// UPT = ceil(nvec * L / EPT / NT) work units per thread.
//   tw[k * twstep] = exp(-2 pi i k / L), k in [0, L)
//   nzero: input elements k >= nzero are taken as zero without reading LDS
//   ld(v, k, x): applied to every input element read in the first pass
//   keep(v, k): output element k of vector v is stored only if true
template <typename T, int L, int EPT, int DIR, int UPT>
struct LdsFft {
  static_assert(EPT <= 16 && (EPT & (EPT - 1)) == 0, "EPT must be a power of two <= 16");
  static_assert(L >= EPT && L % EPT == 0, "bad FFT length");
  static constexpr int TPV = L / EPT;

  cx<T>* buf;
  int nvec, vstride, estride;
  const cx<T>* tw;
  int twstep;

  template <int R, int NS, class LoadOp, class KeepOp>
  __device__ __forceinline__ void pass(int nzero, const LoadOp& ld, const KeepOp& keep) {
    constexpr bool FIRST = (NS == 1);
    constexpr bool LAST = (NS * R == L);
    constexpr int BPT = EPT / R;
    constexpr int LR = L / R;
    cx<T> v[UPT][EPT];
    int vec[UPT], tt[UPT];
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      const int unit = threadIdx.x + q * blockDim.x;
      vec[q] = unit % nvec;
      tt[q] = unit / nvec;
      if (tt[q] < TPV) {
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
          const int j = tt[q] + u * TPV;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int k = j + r * LR;
            cx<T> x;
            if (FIRST && k >= nzero) {
              x = cx<T>{T(0), T(0)};
            } else {
              x = buf[vec[q] * vstride + k * estride];
              if (FIRST) x = ld(vec[q], k, x);
            }
            if (NS > 1 && r > 0) {
              const int idx = (j % NS) * r * (L / (NS * R));
              cx<T> w = tw[idx * twstep];
              if (DIR > 0) w.y = -w.y;
              x = x * w;
            }
            v[q][u * R + r] = x;
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      if (tt[q] < TPV) {
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
          fft_reg<T, R, DIR>(&v[q][u * R]);
          const int j = tt[q] + u * TPV;
          const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int k = base + r * NS;
            if (!LAST || keep(vec[q], k)) buf[vec[q] * vstride + k * estride] = v[q][u * R + r];
          }
        }
      }
    }
    __syncthreads();
  }

  template <int NS, class LoadOp, class KeepOp>
  __device__ __forceinline__ void run_from(int nzero, const LoadOp& ld, const KeepOp& keep) {
    constexpr int R = (L / NS < EPT) ? (L / NS) : EPT;
    pass<R, NS>(nzero, ld, keep);
    if constexpr (NS * R < L) run_from<NS * R>(nzero, ld, keep);
  }

  template <class LoadOp = NoLoad, class KeepOp = KeepAll>
  __device__ __forceinline__ void run(int nzero = L, const LoadOp& ld = LoadOp(),
                                      const KeepOp& keep = KeepOp()) {
    run_from<1>(nzero, ld, keep);
  }
};

template <int a, int b>
struct CeilDiv {
  static constexpr int value = (a + b - 1) / b;
};

}  // namespace pdfk
