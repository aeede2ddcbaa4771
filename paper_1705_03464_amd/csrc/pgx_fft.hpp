// Line FFTs for gfx950: complex arithmetic, in-register DFTs of size <= 32 and
// a multi-stage Stockham transform of one grid line held across a group of
// threads (each thread keeps E elements in registers, stages exchange through
// LDS).  Used by every transform pass of the pair-galaxy correlation.
//
// Conventions: forward DFT X[k] = sum_n x[n] exp(-2 pi i k n / N) (DIR = -1),
// inverse X[k] = sum_n x[n] exp(+2 pi i k n / N) (DIR = +1, unnormalised).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pgx {

template <typename T> struct C { T x, y; };

template <typename T> __device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ C<T> cmulc(C<T> a, C<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// cos(2 pi k / 32) for k = 0..8; other angles follow by quadrant symmetry.
__host__ __device__ constexpr double kCos32(int k) {
  return k == 0 ? 1.0 : k == 1 ? 0.9807852804032304 : k == 2 ? 0.9238795325112867
       : k == 3 ? 0.8314696123025452 : k == 4 ? 0.7071067811865476 : k == 5 ? 0.5555702330196023
       : k == 6 ? 0.38268343236508984 : k == 7 ? 0.19509032201612833 : 0.0;
}
// (cos, sin) of 2 pi e / 32 for any e in [0, 32)
__host__ __device__ constexpr double cos32(int e) {
  return (e / 8) == 0 ? kCos32(e % 8) : (e / 8) == 1 ? -kCos32(8 - e % 8)
       : (e / 8) == 2 ? -kCos32(e % 8) : kCos32(8 - e % 8);
}
__host__ __device__ constexpr double sin32(int e) {
  return (e / 8) == 0 ? kCos32(8 - e % 8) : (e / 8) == 1 ? kCos32(e % 8)
       : (e / 8) == 2 ? -kCos32(8 - e % 8) : -kCos32(e % 8);
}

// v * exp(DIR * 2 pi i * E / R) with E, R compile-time (R a power of two <= 32)
template <int R, int E, int DIR, typename T>
__device__ __forceinline__ C<T> twc(C<T> v) {
  constexpr int e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (2 * e == R) {
    return {-v.x, -v.y};
  } else if constexpr (4 * e == R) {  // exp(DIR * i pi / 2) = DIR * i
    return DIR < 0 ? C<T>{v.y, -v.x} : C<T>{-v.y, v.x};
  } else if constexpr (4 * e == 3 * R) {
    return DIR < 0 ? C<T>{-v.y, v.x} : C<T>{v.y, -v.x};
  } else {
    constexpr int e32 = e * (32 / R);
    constexpr T c = (T)cos32(e32);
    constexpr T s = (T)(DIR * sin32(e32));
    return {v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

template <int DIR, typename T>
__device__ __forceinline__ void bfly4(C<T>& a0, C<T>& a1, C<T>& a2, C<T>& a3) {
  C<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  // DIR * i * t3
  C<T> r3 = DIR < 0 ? C<T>{t3.y, -t3.x} : C<T>{-t3.y, t3.x};
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, r3);
  a3 = csub(t1, r3);
}

// In-register DFT of size R (power of two <= 32), natural order in and out.
template <int R, int DIR, typename T> struct Dft;

template <int R, int DIR, typename T, int K> struct R4Combine {
  __device__ __forceinline__ static void run(C<T> (&y)[4][R / 4], C<T>* x) {
    constexpr int M = R / 4;
    if constexpr (K < M) {
      C<T> a0 = y[0][K];
      C<T> a1 = twc<R, K, DIR>(y[1][K]);
      C<T> a2 = twc<R, 2 * K, DIR>(y[2][K]);
      C<T> a3 = twc<R, 3 * K, DIR>(y[3][K]);
      bfly4<DIR>(a0, a1, a2, a3);
      x[K] = a0;
      x[K + M] = a1;
      x[K + 2 * M] = a2;
      x[K + 3 * M] = a3;
      R4Combine<R, DIR, T, K + 1>::run(y, x);
    }
  }
};

template <int R, int DIR, typename T> struct Dft {
  __device__ __forceinline__ static void run(C<T>* x) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
      C<T> a = x[0], b = x[1];
      x[0] = cadd(a, b);
      x[1] = csub(a, b);
    } else if constexpr (R == 4) {
      bfly4<DIR>(x[0], x[1], x[2], x[3]);
    } else {
      constexpr int M = R / 4;
      C<T> y[4][M];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < M; ++m) y[q][m] = x[4 * m + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) Dft<M, DIR, T>::run(y[q]);
      R4Combine<R, DIR, T, 0>::run(y, x);
    }
  }
};

// ---------------------------------------------------------------------------
// Stage shapes of the Stockham line transform.  R0 = E = elements per thread;
// later radices divide E.  Threads per line TPL = N / E.
// ---------------------------------------------------------------------------
template <int N, int S, int R0, int R1, int R2> struct Shape {
  static constexpr int n = N, stages = S, E = R0, TPL = N / R0;
  static constexpr int radix(int s) { return s == 0 ? R0 : s == 1 ? R1 : R2; }
  static constexpr int ns(int s) { return s == 0 ? 1 : s == 1 ? R0 : R0 * R1; }
  // twiddle tables: stage s >= 1 has Ns * R entries exp(-2 pi i r k / (Ns R)),
  // stored at [twoff(s) + r * Ns + k] so consecutive k are consecutive entries
  static constexpr int twoff(int s) { return s <= 1 ? 0 : R0 * R1; }
  static constexpr int tw_entries() { return S == 2 ? N : R0 * R1 + N; }
};

template <typename T, int N> struct DefaultShape;
template <> struct DefaultShape<float, 64> { using type = Shape<64, 2, 8, 8, 1>; };
template <> struct DefaultShape<float, 128> { using type = Shape<128, 3, 8, 8, 2>; };
template <> struct DefaultShape<float, 256> { using type = Shape<256, 3, 8, 8, 4>; };
template <> struct DefaultShape<float, 512> { using type = Shape<512, 3, 8, 8, 8>; };
template <> struct DefaultShape<float, 1024> { using type = Shape<1024, 3, 16, 8, 8>; };
template <> struct DefaultShape<double, 64> { using type = Shape<64, 2, 8, 8, 1>; };
template <> struct DefaultShape<double, 128> { using type = Shape<128, 3, 8, 8, 2>; };
template <> struct DefaultShape<double, 256> { using type = Shape<256, 3, 8, 8, 4>; };
template <> struct DefaultShape<double, 512> { using type = Shape<512, 3, 8, 8, 8>; };
template <> struct DefaultShape<double, 1024> { using type = Shape<1024, 3, 16, 8, 8>; };

// Second radix schedule of the strided passes, one of the candidates the
// plan's autotuner times: 16 elements per thread, fewer exchange stages.
template <typename T, int N> struct AltShape;
template <> struct AltShape<float, 64> { using type = Shape<64, 2, 16, 4, 1>; };
template <> struct AltShape<float, 128> { using type = Shape<128, 2, 16, 8, 1>; };
template <> struct AltShape<float, 256> { using type = Shape<256, 2, 16, 16, 1>; };
template <> struct AltShape<float, 512> { using type = Shape<512, 3, 16, 8, 4>; };
template <> struct AltShape<float, 1024> { using type = Shape<1024, 3, 16, 16, 4>; };
template <int N> struct AltShape<double, N> { using type = typename DefaultShape<double, N>::type; };

// LDS index with one pad element per 2^kPadShift (breaks power-of-two strides
// inside a line); kLineExtra sets the line length modulo the bank count so
// the lines of a tile start on different banks.
constexpr int kPadShift = 4;
constexpr int kLineExtra = 1;
__device__ __forceinline__ int lpad(int i) { return i + (i >> kPadShift); }
template <int N> constexpr int lds_line_elems() { return N + (N >> kPadShift) + kLineExtra; }

// Twiddle providers for stage s >= 1 of butterfly q (j = t + TPL*q), radix
// index r, k = j mod Ns: exp(-2 pi i r k / (Ns R)).
//  TwLds  reads the per-stage table from LDS on every use;
//  TwReg  holds this thread's twiddles in registers (loaded once per kernel
//         from the global table); k depends only on t and q, so a thread that
//         transforms many lines reuses them.
template <typename Sh, typename T> struct TwLds {
  const C<T>* tw;
  template <int s> __device__ __forceinline__ C<T> get(int q, int r, int k) const {
    const C<T>* b = tw + k;  // thread base; the stage/radix part is an immediate offset
    return b[Sh::twoff(s) + r * Sh::ns(s)];
  }
};

template <typename Sh, typename T> struct TwReg {
  static constexpr int NS = Sh::stages > 1 ? Sh::stages - 1 : 1;
  C<T> w[NS][Sh::E];
  __device__ __forceinline__ void load(const C<T>* __restrict__ tw_g, int t) {
    load_stage<1>(tw_g, t);
    if constexpr (Sh::stages == 3) load_stage<2>(tw_g, t);
  }
  template <int s> __device__ __forceinline__ void load_stage(const C<T>* __restrict__ tw_g, int t) {
    constexpr int R = Sh::radix(s), Ns = Sh::ns(s), Q = Sh::E / R;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int k = (t + Sh::TPL * q) % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) w[s - 1][q * R + r] = tw_g[Sh::twoff(s) + r * Ns + k];
    }
  }
  template <int s> __device__ __forceinline__ C<T> get(int q, int r, int) const {
    return w[s - 1][q * Sh::radix(s) + r];
  }
};

// One Stockham stage for the butterflies owned by thread t (j = t + TPL*q).
// `in` values are in registers (stage 0) or read from LDS (later stages).
template <typename Sh, int s, int DIR, typename T, typename TW>
__device__ __forceinline__ void stage_compute(C<T>* v, int t, const TW& tw) {
  constexpr int E = Sh::E, TPL = Sh::TPL;
  constexpr int R = Sh::radix(s), Ns = Sh::ns(s), Q = E / R;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    C<T>* b = v + q * R;
    if constexpr (Ns > 1) {
      const int j = t + TPL * q;
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C<T> w = tw.template get<s>(q, r, k);
        if constexpr (DIR > 0) w.y = -w.y;
        b[r] = cmul(b[r], w);
      }
    }
    Dft<R, DIR, T>::run(b);
  }
}

// The exchanges address the line at lpad(B + K), B depending on the thread,
// K a compile-time constant.  lpad(B + K) = lpad(B) + K + (K >> kPadShift)
// whenever (B mod P) + (K mod P) < P (P = 2^kPadShift): then every access of a
// thread is one base address plus an immediate offset.  pad_linear<Sh>()
// checks that condition for all threads and accesses of a shape.
template <typename Sh> constexpr bool pad_linear() {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, P = 1 << kPadShift;
  for (int t = 0; t < TPL; ++t) {
    for (int r = 0; r < E; ++r)  // stage-0 outputs: B = t E, K = r
      if ((t * E) % P + r % P >= P) return false;
    for (int s = 1; s < Sh::stages; ++s) {  // stage inputs: B = t, K = TPL q + r N / R
      const int R = Sh::radix(s), Q = E / R;
      for (int q = 0; q < Q; ++q)
        for (int r = 0; r < R; ++r)
          if (t % P + (TPL * q + r * (N / R)) % P >= P) return false;
    }
    if (Sh::stages == 3) {  // stage-1 outputs: B = (t/Ns) Ns R + t % Ns, K = TPL q R + r Ns
      const int R = Sh::radix(1), Ns = Sh::ns(1), Q = E / R;
      if (TPL % Ns != 0) return false;
      const int B = (t / Ns) * Ns * R + t % Ns;
      for (int q = 0; q < Q; ++q)
        for (int r = 0; r < R; ++r)
          if (B % P + (TPL * q * R + r * Ns) % P >= P) return false;
    }
  }
  return true;
}

// Full line transform.  On entry v[m] holds element t + TPL*m of the line; on
// exit v[m] holds output element t + TPL*m.  `line` is this line's LDS buffer
// (lds_line_elems<N>() entries); `tw` the per-stage forward twiddle tables in LDS.
// SYNC is a callable that synchronises all threads sharing `line`.
template <typename Sh, int DIR, typename T, typename Sync, typename TW>
__device__ __forceinline__ void line_fft_tw(C<T>* v, int t, C<T>* line, const TW& tw, Sync sync) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL;
  constexpr bool LIN = pad_linear<Sh>();
  // stage 0: inputs j + r*(N/R0) with j = t  ->  v[r] already in place
  stage_compute<Sh, 0, DIR, T, TW>(v, t, tw);
  if constexpr (Sh::stages == 1) return;
  // write stage-0 outputs: (j/Ns)*Ns*R + j%Ns + r*Ns with Ns = 1 -> j*R0 + r
  {
    C<T>* lw = line + lpad(t * E);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      if constexpr (LIN) lw[r + (r >> kPadShift)] = v[r];
      else line[lpad(t * E + r)] = v[r];
    }
  }
  sync();
  C<T>* lr = line + lpad(t);  // base of every stage's inputs
  {
    constexpr int R = Sh::radix(1), Q = E / R;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int K = TPL * q + r * (N / R);
        if constexpr (LIN) v[q * R + r] = lr[K + (K >> kPadShift)];
        else v[q * R + r] = line[lpad(t + K)];
      }
  }
  stage_compute<Sh, 1, DIR, T, TW>(v, t, tw);
  if constexpr (Sh::stages == 3) {
    constexpr int R = Sh::radix(1), Ns = Sh::ns(1), Q = E / R;
    sync();
    if constexpr (LIN) {
      C<T>* lm = line + lpad((t / Ns) * Ns * R + t % Ns);
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int K = TPL * q * R + r * Ns;
          lm[K + (K >> kPadShift)] = v[q * R + r];
        }
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int j = t + TPL * q;
        const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) line[lpad(base + r * Ns)] = v[q * R + r];
      }
    }
    sync();
    constexpr int R2 = Sh::radix(2), Q2 = E / R2;
#pragma unroll
    for (int q = 0; q < Q2; ++q)
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int K = TPL * q + r * (N / R2);
        if constexpr (LIN) v[q * R2 + r] = lr[K + (K >> kPadShift)];
        else v[q * R2 + r] = line[lpad(t + K)];
      }
    stage_compute<Sh, 2, DIR, T, TW>(v, t, tw);
  }
  // last stage: butterfly q, output r -> element j + r*Ns = t + TPL*(q + r*Q);
  // reorder registers to v[m] <-> element t + TPL*m
  {
    constexpr int RL = Sh::radix(Sh::stages - 1), QL = E / RL;
    if constexpr (QL > 1) {
      C<T> tmp[E];
#pragma unroll
      for (int q = 0; q < QL; ++q)
#pragma unroll
        for (int r = 0; r < RL; ++r) tmp[q + r * QL] = v[q * RL + r];
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = tmp[m];
    }
  }
}

// Line transform with the per-stage twiddle table in LDS.
template <typename Sh, int DIR, typename T, typename Sync>
__device__ __forceinline__ void line_fft(C<T>* v, int t, C<T>* line, const C<T>* tw, Sync sync) {
  line_fft_tw<Sh, DIR, T>(v, t, line, TwLds<Sh, T>{tw}, sync);
}

}  // namespace pgx
