// Batched complex FFTs on data resident in LDS, for one workgroup.
//
// Radix-R Stockham autosort passes: each thread holds EPT elements of one
// vector in registers, does EPT/R radix-R butterflies per pass with the
// in-register FFTs below, and exchanges through LDS between passes, either in
// place (load all, barrier, store all, barrier) or between two disjoint
// regions of the tile (load, store, one barrier); no bit reversal is needed.  Vectors are rows or columns of a 2-D tile.  Threads are
// assigned vector-fastest, so neighbouring lanes touch neighbouring rows or
// columns.  Zero-padded inputs and cropped outputs are known at compile time
// and their butterflies are skipped.
//
// Forward transforms use exp(-2 pi i jk/L) (DIR = -1), inverse ones
// exp(+2 pi i jk/L) (DIR = +1); neither is normalised.
#pragma once

#include <type_traits>
#include <utility>

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

// Compile-time loop: f(std::integral_constant<int, i>) for i in [0, N).
template <class F, int... I>
__host__ __device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// v * exp(DIR 2 pi i E / 16) with the trivial and 45-degree rotations spelled
// out (IEEE rules forbid the compiler from folding multiplications by 0 or 1).
template <typename T, int E, int DIR>
__host__ __device__ __forceinline__ cx<T> rot16(cx<T> v) {
  constexpr int e = ((E % 16) + 16) % 16;
  constexpr T h = T(0.70710678118654752440);
  if constexpr (e == 0) {
    return v;
  } else if constexpr (e == 8) {
    return {-v.x, -v.y};
  } else if constexpr (e == 4) {          // exp(DIR i pi/2) = DIR i
    return DIR > 0 ? cx<T>{-v.y, v.x} : cx<T>{v.y, -v.x};
  } else if constexpr (e == 12) {         // -DIR i
    return DIR > 0 ? cx<T>{v.y, -v.x} : cx<T>{-v.y, v.x};
  } else if constexpr (e % 4 == 2) {      // odd multiples of 45 degrees
    constexpr T c = T(cos16(e)), sn = T(DIR * cos16(e - 4));
    // c, sn = +-h: (c x - sn y, sn x + c y) with one add and one multiply per part
    constexpr T sa = c > 0 ? h : -h;
    constexpr T sb = sn > 0 ? h : -h;
    if constexpr (c > 0 && sn > 0) return {h * (v.x - v.y), h * (v.x + v.y)};
    else if constexpr (c > 0 && sn < 0) return {h * (v.x + v.y), h * (v.y - v.x)};
    else if constexpr (c < 0 && sn > 0) return {-h * (v.x + v.y), h * (v.x - v.y)};
    else return {h * (v.y - v.x), -h * (v.x + v.y)};
    (void)sa;
    (void)sb;
  } else {
    constexpr T c = T(cos16(e)), sn = T(DIR * cos16(e - 4));
    return {c * v.x - sn * v.y, sn * v.x + c * v.y};
  }
}

template <int R>
__host__ __device__ constexpr int ilog2(int n) {
  return n <= 1 ? 0 : 1 + ilog2<R>(n / 2);
}

// Zero pattern of the register file before radix-2 stage `st` of fft_reg,
// when inputs r >= ZR are known zeros: bit i set = register i holds zero.
template <int R>
__host__ __device__ constexpr unsigned zero_mask(int ZR, int st) {
  unsigned m = 0;
  for (int i = 0; i < R; ++i)
    if (bitrev<R>(i) >= ZR) m |= 1u << i;
  for (int t = 0; t < st; ++t) {
    const int s = 1 << t;
    unsigned o = m;
    for (int k = 0; k < R; k += 2 * s)
      for (int j = 0; j < s; ++j) {
        const bool z = ((m >> (k + j)) & 1u) && ((m >> (k + j + s)) & 1u);
        o = z ? (o | (1u << (k + j)) | (1u << (k + j + s))) : (o & ~((1u << (k + j)) | (1u << (k + j + s))));
      }
    m = o;
  }
  return m;
}

// In-register FFT of R points (R = 1, 2, 4, 8, 16), natural order in and out:
// bit reversal, then radix-2 decimation-in-time stages, all indices and
// twiddles resolved at compile time.  Inputs r >= ZR are known to be zero
// (their butterflies are skipped) and only outputs r < KR are needed.
template <typename T, int R, int DIR, int ZR = R, int KR = R>
__host__ __device__ __forceinline__ void fft_reg(cx<T>* v);

// cos(2 pi k / 12); sin(2 pi k / 12) = cos(2 pi (k - 3) / 12).
__host__ __device__ constexpr double cos12(int k) {
  switch (((k % 12) + 12) % 12) {
    case 0: return 1.0;
    case 1: return 0.86602540378443864676;
    case 2: return 0.5;
    case 3: return 0.0;
    case 4: return -0.5;
    case 5: return -0.86602540378443864676;
    case 6: return -1.0;
    case 7: return -0.86602540378443864676;
    case 8: return -0.5;
    case 9: return 0.0;
    case 10: return 0.5;
    default: return 0.86602540378443864676;
  }
}

// v * exp(DIR 2 pi i E / 12), trivial rotations spelled out
template <typename T, int E, int DIR>
__host__ __device__ __forceinline__ cx<T> rot12(cx<T> v) {
  constexpr int e = ((E % 12) + 12) % 12;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (e == 6) {
    return {-v.x, -v.y};
  } else if constexpr (e == 3) {
    return DIR > 0 ? cx<T>{-v.y, v.x} : cx<T>{v.y, -v.x};
  } else if constexpr (e == 9) {
    return DIR > 0 ? cx<T>{v.y, -v.x} : cx<T>{-v.y, v.x};
  } else {
    constexpr T c = T(cos12(e)), sn = T(DIR * cos12(e - 3));
    return {c * v.x - sn * v.y, sn * v.x + c * v.y};
  }
}

// 3-point DFT in place: (a, b, c) -> (a + b + c, a + w b + w^2 c, a + w^2 b + w c), w = exp(DIR 2 pi i / 3)
template <typename T, int DIR>
__host__ __device__ __forceinline__ void dft3(cx<T>& a, cx<T>& b, cx<T>& c) {
  const cx<T> s = b + c, d = b - c;
  const cx<T> m{a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
  const T k = T(DIR * 0.86602540378443864676);
  const cx<T> id{-k * d.y, k * d.x};  // i k d
  a = a + s;
  b = m + id;
  c = m - id;
}

// In-register DFT of R = 3 Q points (Q = 1, 2, 4), natural order in and out:
// with n = Q n1 + n2 and k = k1 + 3 k2,
//   X[k1 + 3 k2] = sum_n2 W_Q^{n2 k2} W_R^{n2 k1} sum_n1 x[Q n1 + n2] W_3^{n1 k1},
// i.e. 3-point DFTs across the stride Q, the twiddles W_R^{n2 k1}, and Q-point
// FFTs of each k1 row; the final relabelling of registers is free.
template <typename T, int R, int DIR>
__host__ __device__ __forceinline__ void fft_mixed(cx<T>* v) {
  constexpr int Q = R / 3;
  static_assert(R == 3 * Q && (Q == 1 || Q == 2 || Q == 4), "radix 3, 6 or 12");
  static_for<Q>([&](auto n2c) {
    constexpr int n2 = decltype(n2c)::value;
    dft3<T, DIR>(v[n2], v[Q + n2], v[2 * Q + n2]);  // output k1 at v[Q k1 + n2]
  });
  static_for<Q>([&](auto n2c) {
    constexpr int n2 = decltype(n2c)::value;
    v[Q + n2] = rot12<T, n2 * 1 * (12 / R), DIR>(v[Q + n2]);
    v[2 * Q + n2] = rot12<T, n2 * 2 * (12 / R), DIR>(v[2 * Q + n2]);
  });
  if constexpr (Q > 1) {
    fft_reg<T, Q, DIR>(&v[0]);
    fft_reg<T, Q, DIR>(&v[Q]);
    fft_reg<T, Q, DIR>(&v[2 * Q]);
  }
  cx<T> t[R];
  static_for<R>([&](auto ic) {
    constexpr int i = decltype(ic)::value;  // i = Q k1 + k2  ->  output k1 + 3 k2
    t[(i / Q) + 3 * (i % Q)] = v[i];
  });
  static_for<R>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    v[i] = t[i];
  });
}

template <typename T, int R, int DIR, int ZR, int KR>
__host__ __device__ __forceinline__ void fft_reg(cx<T>* v) {
  if constexpr (R % 3 == 0) {
    fft_mixed<T, R, DIR>(v);  // no pruning: zero inputs are loaded as zeros, unused outputs not stored
  } else if constexpr (R > 1) {
    static_for<R>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      constexpr int j = bitrev<R>(i);
      if constexpr (j > i) {
        cx<T> t = v[i];
        v[i] = v[j];
        v[j] = t;
      }
    });
    constexpr int L2 = ilog2<R>(R);
    static_for<L2>([&](auto stc) {
      constexpr int st = decltype(stc)::value;
      constexpr int s = 1 << st;
      constexpr unsigned zm = zero_mask<R>(ZR, st);
      constexpr bool last = st == L2 - 1;
      static_for<R / 2>([&](auto bc) {
        constexpr int bidx = decltype(bc)::value;
        constexpr int k = (bidx / s) * 2 * s, j = bidx % s;
        constexpr bool za = (zm >> (k + j)) & 1u, zb = (zm >> (k + j + s)) & 1u;
        constexpr bool lo = !last || (k + j) < KR, hi = !last || (k + j + s) < KR;
        if constexpr (za && zb) {
          // both inputs are zero registers: so are both outputs
        } else if constexpr (zb) {
          if constexpr (hi) v[k + j + s] = v[k + j];
        } else if constexpr (za) {
          const cx<T> b = rot16<T, j * (16 / (2 * s)), DIR>(v[k + j + s]);
          if constexpr (lo) v[k + j] = b;
          if constexpr (hi) v[k + j + s] = cx<T>{-b.x, -b.y};
        } else {
          const cx<T> a = v[k + j];
          const cx<T> b = rot16<T, j * (16 / (2 * s)), DIR>(v[k + j + s]);
          if constexpr (lo) v[k + j] = a + b;
          if constexpr (hi) v[k + j + s] = a - b;
        }
      });
    });
  }
}

struct NoLoad {
  template <typename C>
  __device__ __forceinline__ C operator()(int, int, C v) const { return v; }
};

// Orders LDS accesses of one wavefront (its lanes exchange data through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Layout of a P-wide complex tile in LDS: element (i, c) at i * (P + 1) + c.
// LDS serves 16 lanes of an 8-byte access per cycle from 32 four-byte banks;
// the odd row stride sends 16 consecutive rows at one column, and 16
// consecutive columns of one row, to 16 different bank pairs.
template <int P>
struct Tile {
  static constexpr int LD = P + 1;
  __device__ __forceinline__ static int at(int i, int c) { return i * LD + c; }
};

// Vectors of a tile: rows (element k = column k) or columns (element k = row
// k).  NV is the compile-time vector count; a mapped set holds nv <= NV
// vectors, vector v being row / column (kmin + v) mod NV (the kept Fourier
// modes of a centred or corner set).
template <int P, int NV_, bool ROWS, bool MAPPED = false, bool WAVE_LOCAL = false>
struct Vecs {
  static constexpr int NV = NV_;
  // wave-local: a vector's threads sit in one wavefront (numbered
  // vector-fastest inside it) and passes synchronise only the wavefront;
  // otherwise threads are numbered vector-fastest across the workgroup and
  // passes use workgroup barriers
  static constexpr bool WL = WAVE_LOCAL;
  int nv = NV_;
  int kmin = 0;
  __device__ __forceinline__ int addr(int v, int k) const {
    int x = v;
    if constexpr (MAPPED) {
      x = kmin + v;  // kmin in (-NV, 0] and v < NV: one wrap suffices
      if constexpr ((NV & (NV - 1)) == 0)
        x &= NV - 1;
      else
        x += x < 0 ? NV : 0;
    }
    return ROWS ? Tile<P>::at(x, k) : Tile<P>::at(k, x);
  }
};

// Radix-R Stockham passes (R <= 16) over the vectors of a Vecs set, L points
// each, EPT elements per thread, NT threads.  tw[k * TWS] = exp(-2 pi i k / L).
// After a wave-local transform, callers put a workgroup barrier before any
// phase that reads another wavefront's vectors.
template <typename T, int L, int EPT, int NT, class V, int TWS>
struct Fft {
  static_assert(EPT <= 32, "at most 32 elements per thread");
  static_assert(L >= EPT && L % EPT == 0, "bad FFT length");
  static constexpr int TPV = L / EPT;
  static constexpr int UPT = (V::NV * TPV + NT - 1) / NT;
  static_assert(!V::WL || (64 % TPV == 0 && NT % 64 == 0), "a vector's threads must sit in one wavefront");
  static constexpr int VPW = 64 / TPV;  // vectors per wavefront (wave-local sets)

  __device__ __forceinline__ static void sync() {
    if constexpr (V::WL)
      wave_sync();
    else
      __syncthreads();
  }

  cx<T>* buf;
  const cx<T>* tw;
  V vs;

  // radix of the pass at stride NS: the largest of 16, 12, 8, 6, 4, 3, 2 that
  // divides both the remaining length and the elements per thread
  __host__ __device__ static constexpr int radix(int NS) {
    constexpr int cand[7] = {16, 12, 8, 6, 4, 3, 2};
    for (int r : cand)
      if (r <= EPT && (L / NS) % r == 0 && EPT % r == 0) return r;
    return 0;  // no plan: rejected by the asserts of the pass
  }

  struct Regs {
    cx<T> v[UPT][EPT];
    int vec[UPT], t[UPT];
    bool act[UPT];
  };

  __device__ __forceinline__ void assign(Regs& g) const {
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      const int unit = threadIdx.x + q * NT;
      if constexpr (V::WL) {
        const int lane = unit & 63;
        g.vec[q] = (unit >> 6) * VPW + lane % VPW;
        g.t[q] = lane / VPW;
      } else {
        g.vec[q] = unit % V::NV;
        g.t[q] = unit / V::NV;
      }
      g.act[q] = g.vec[q] < vs.nv && g.t[q] < TPV;
    }
  }

  // Load of a pass: element j + r L/R of the butterflies j = t + u TPV, with
  // the pass twiddle.  In a first pass (NS = 1) inputs r >= ZR are zero and
  // ld(v, k, x) is applied to every element read.
  template <int R, int NS, int DIR, int ZR, class LoadOp>
  __device__ __forceinline__ void load(Regs& g, const LoadOp& ld, int off = 0) const {
    constexpr int BPT = EPT / R, LR = L / R;
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      if (!g.act[q]) continue;
#pragma unroll
      for (int u = 0; u < BPT; ++u) {
        const int j = g.t[q] + u * TPV;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cx<T> x{T(0), T(0)};
          if (r < ZR) {
            const int k = j + r * LR;
            x = buf[off + vs.addr(g.vec[q], k)];
            if constexpr (NS == 1) x = ld(g.vec[q], k, x);
            if constexpr (NS > 1) {
              if (r > 0) {
                cx<T> w = tw[((j % NS) * r * (L / (NS * R))) * TWS];
                if (DIR > 0) w.y = -w.y;
                x = x * w;
              }
            }
          }
          g.v[q][u * R + r] = x;
        }
      }
    }
  }

  template <int R, int DIR, int ZR, int KR>
  __device__ __forceinline__ void compute(Regs& g) const {
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      if (!g.act[q]) continue;
#pragma unroll
      for (int u = 0; u < EPT / R; ++u) fft_reg<T, R, DIR, ZR, KR>(&g.v[q][u * R]);
    }
  }

  // Store of a pass: output r of butterfly j goes to (j / NS) NS R + j % NS + r NS;
  // only outputs r < KR are written.
  template <int R, int NS, int KR>
  __device__ __forceinline__ void store(const Regs& g, int off = 0) const {
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      if (!g.act[q]) continue;
#pragma unroll
      for (int u = 0; u < EPT / R; ++u) {
        const int j = g.t[q] + u * TPV;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < KR; ++r) buf[off + vs.addr(g.vec[q], base + r * NS)] = g.v[q][u * R + r];
      }
    }
  }

  // One full pass in place on the region at element offset off: load,
  // barrier, butterflies, store, barrier.
  template <int R, int NS, int DIR, int ZR, int KR, class LoadOp>
  __device__ __forceinline__ void pass(const LoadOp& ld, int off = 0) const {
    Regs g;
    assign(g);
    load<R, NS, DIR, ZR>(g, ld, off);
    sync();
    compute<R, DIR, ZR, KR>(g);
    store<R, NS, KR>(g, off);
    sync();
  }

  // One pass from region src to the disjoint region dst (element offsets into
  // the tile): loads, butterflies, stores, then one barrier; no barrier is
  // needed between the loads and the stores.
  template <int R, int NS, int DIR, int ZR, int KR, class LoadOp>
  __device__ __forceinline__ void pass_oop(const LoadOp& ld, int src, int dst) const {
    Regs g;
    assign(g);
    load<R, NS, DIR, ZR>(g, ld, src);
    compute<R, DIR, ZR, KR>(g);
    store<R, NS, KR>(g, dst);
    sync();
  }

  // The whole transform alternating between the disjoint regions a and b (the
  // first pass reads a); returns the offset of the region holding the result.
  template <int DIR, int NZ = L, int KEEP = L, int NS = 1, class LoadOp = NoLoad>
  __device__ __forceinline__ int run_pp(int a, int b, const LoadOp& ld = LoadOp()) const {
    constexpr int R = radix(NS);
    constexpr bool first = NS == 1, last = NS * R == L;
    constexpr int ZR = first ? (NZ * R + L - 1) / L : R;
    constexpr int KR = last ? (KEEP + NS - 1) / NS : R;
    static_assert(!first || (NZ * R) % L == 0, "zero prefix must align with the first pass");
    static_assert(!last || KEEP % NS == 0, "kept prefix must align with the last pass");
    pass_oop<R, NS, DIR, ZR, KR>(ld, a, b);
    if constexpr (!last)
      return run_pp<DIR, NZ, KEEP, NS * R>(b, a, ld);
    else
      return b;
  }

  // The whole transform with radices EPT, EPT, ..., remainder.  NZ: inputs
  // k >= NZ are zero; KEEP: only outputs k < KEEP are stored (both must be
  // multiples of the stride they apply at, e.g. L/2).
  template <int DIR, int NZ = L, int KEEP = L, int NS = 1, class LoadOp = NoLoad>
  __device__ __forceinline__ void run(const LoadOp& ld = LoadOp(), int off = 0) const {
    constexpr int R = radix(NS);
    constexpr bool first = NS == 1, last = NS * R == L;
    constexpr int ZR = first ? (NZ * R + L - 1) / L : R;
    constexpr int KR = last ? (KEEP + NS - 1) / NS : R;
    static_assert(!first || (NZ * R) % L == 0, "zero prefix must align with the first pass");
    static_assert(!last || KEEP % NS == 0, "kept prefix must align with the last pass");
    pass<R, NS, DIR, ZR, KR>(ld, off);
    if constexpr (!last) run<DIR, NZ, KEEP, NS * R>(ld, off);
  }
};

template <int a, int b>
struct CeilDiv {
  static constexpr int value = (a + b - 1) / b;
};

}  // namespace pdfk
