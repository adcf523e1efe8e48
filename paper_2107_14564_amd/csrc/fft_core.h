// Device-side building blocks of the hand-written FFTs: complex helpers, small
// DFT butterflies and an in-place Stockham (self-sorting) pass sequence over a
// batch of lines held in LDS.
//
// Stockham autosort, radix-R pass with current span ns (product of the radices
// already applied, starting at 1): butterfly j (0 <= j < n/R) reads
// v_r = x[j + r n/R], multiplies v_r by W_{ns R}^{r (j mod ns)}, takes an
// R-point DFT and writes it to y[(j div ns) ns R + (j mod ns) + r ns].  After
// the last pass ns = n and y holds the DFT in natural order.  Each pass is done
// in place: every thread first loads all elements of its butterflies into
// registers, the work group synchronises, then all threads store.  Line
// length, radix schedule and tile shape are compile-time constants, so all
// index arithmetic reduces to shifts and constant multiplies.
#pragma once

#include <hip/hip_runtime.h>

namespace bispec {

template <typename T> struct V2t;
template <> struct V2t<float> { using type = float2; };
template <> struct V2t<double> { using type = double2; };
template <typename T> using V2 = typename V2t<T>::type;

template <typename T> __device__ __forceinline__ V2<T> mk(T x, T y) { V2<T> r; r.x = x; r.y = y; return r; }
template <typename T> __device__ __forceinline__ V2<T> add(V2<T> a, V2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ V2<T> sub(V2<T> a, V2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ V2<T> mul(V2<T> a, V2<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ V2<T> conjv(V2<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ V2<T> scl(V2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by sign*i (sign = +1 or -1)
template <typename T> __device__ __forceinline__ V2<T> mul_i(V2<T> a, T sign) { return mk<T>(-sign * a.y, sign * a.x); }

// In-register R-point DFT, out[q] = sum_r in[r] exp(sign 2 pi i r q / R).
template <typename T, int R> struct Dft;

template <typename T> struct Dft<T, 2> {
  __device__ __forceinline__ static void run(V2<T>* v, T) {
    V2<T> a = v[0], b = v[1];
    v[0] = add<T>(a, b);
    v[1] = sub<T>(a, b);
  }
};

template <typename T> struct Dft<T, 4> {
  __device__ __forceinline__ static void run(V2<T>* v, T sign) {
    V2<T> s02 = add<T>(v[0], v[2]), d02 = sub<T>(v[0], v[2]);
    V2<T> s13 = add<T>(v[1], v[3]), d13 = mul_i<T>(sub<T>(v[1], v[3]), sign);
    v[0] = add<T>(s02, s13);
    v[2] = sub<T>(s02, s13);
    v[1] = add<T>(d02, d13);
    v[3] = sub<T>(d02, d13);
  }
};

template <typename T> struct Dft<T, 8> {
  __device__ __forceinline__ static void run(V2<T>* v, T sign) {
    // two radix-4 DFTs on even and odd samples, then combine with W8^q
    V2<T> e[4] = {v[0], v[2], v[4], v[6]};
    V2<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4>::run(e, sign);
    Dft<T, 4>::run(o, sign);
    const T h = (T)0.70710678118654752440084436210484903928;
    // W8^1 = (1 + sign i) h, W8^2 = sign i, W8^3 = (-1 + sign i) h
    V2<T> o1 = mk<T>(h * (o[1].x - sign * o[1].y), h * (o[1].y + sign * o[1].x));
    V2<T> o2 = mul_i<T>(o[2], sign);
    V2<T> o3 = mk<T>(h * (-o[3].x - sign * o[3].y), h * (-o[3].y + sign * o[3].x));
    v[0] = add<T>(e[0], o[0]);
    v[4] = sub<T>(e[0], o[0]);
    v[1] = add<T>(e[1], o1);
    v[5] = sub<T>(e[1], o1);
    v[2] = add<T>(e[2], o2);
    v[6] = sub<T>(e[2], o2);
    v[3] = add<T>(e[3], o3);
    v[7] = sub<T>(e[3], o3);
  }
};

template <typename T> struct Dft<T, 3> {
  __device__ __forceinline__ static void run(V2<T>* v, T sign) {
    const T c = (T)-0.5, s = sign * (T)0.86602540378443864676372317075293618347;
    V2<T> a = v[0], b = v[1], d = v[2];
    V2<T> t = add<T>(b, d);
    V2<T> u = sub<T>(b, d);
    V2<T> m = mk<T>(a.x + c * t.x, a.y + c * t.y);
    V2<T> r = mk<T>(-s * u.y, s * u.x);
    v[0] = add<T>(a, t);
    v[1] = add<T>(m, r);
    v[2] = sub<T>(m, r);
  }
};

template <typename T> struct Dft<T, 5> {
  __device__ __forceinline__ static void run(V2<T>* v, T sign) {
    const T c1 = (T)0.30901699437494742410229341718281905886;   // cos(2pi/5)
    const T c2 = (T)-0.80901699437494742410229341718281905886;  // cos(4pi/5)
    const T s1 = sign * (T)0.95105651629515357211643933337938214340;  // sin(2pi/5)
    const T s2 = sign * (T)0.58778525229247312916870595463907276860;  // sin(4pi/5)
    V2<T> a = v[0];
    V2<T> t1 = add<T>(v[1], v[4]), u1 = sub<T>(v[1], v[4]);
    V2<T> t2 = add<T>(v[2], v[3]), u2 = sub<T>(v[2], v[3]);
    V2<T> m1 = mk<T>(a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y);
    V2<T> m2 = mk<T>(a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y);
    // i * (s1 u1 + s2 u2) and i * (s2 u1 - s1 u2)
    V2<T> r1 = mk<T>(-(s1 * u1.y + s2 * u2.y), s1 * u1.x + s2 * u2.x);
    V2<T> r2 = mk<T>(-(s2 * u1.y - s1 * u2.y), s2 * u1.x - s1 * u2.x);
    v[0] = add<T>(a, add<T>(t1, t2));
    v[1] = add<T>(m1, r1);
    v[4] = sub<T>(m1, r1);
    v[2] = add<T>(m2, r2);
    v[3] = sub<T>(m2, r2);
  }
};

// Composite radix R = R1 R2 in registers (one LDS pass instead of two):
// with r = R2 a + b and q = c + R1 d, out[c + R1 d] = sum_b W_R2^(b d)
// [W_R^(b c) sum_a in[R2 a + b] W_R1^(a c)]: R1-point DFTs over a for each b,
// the twiddles W_R^(b c), then R2-point DFTs over b for each c.
// exp(sign 2 pi i m / R) for the twiddles, as (cos, sin) with the sign applied
template <typename T>
__device__ __forceinline__ V2<T> rot(V2<T> x, T c, T s, T sign) {
  return mk<T>(x.x * c - sign * s * x.y, x.y * c + sign * s * x.x);
}

template <typename T> struct Dft<T, 16> {
  __device__ __forceinline__ static void run(V2<T>* v, T sign) {
    const T c1 = (T)0.92387953251128675612818318939678828682;  // cos(pi/8)
    const T s1 = (T)0.38268343236508977172845998403039886676;  // sin(pi/8)
    const T h = (T)0.70710678118654752440084436210484903928;   // cos(pi/4)
    V2<T> y[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      V2<T> t[4] = {v[b], v[b + 4], v[b + 8], v[b + 12]};
      Dft<T, 4>::run(t, sign);
#pragma unroll
      for (int c = 0; c < 4; ++c) y[b][c] = t[c];
    }
    // W_16^(b c): m = 1, 2, 3, 2, 4, 6, 3, 6, 9
    y[1][1] = rot<T>(y[1][1], c1, s1, sign);
    y[1][2] = rot<T>(y[1][2], h, h, sign);
    y[1][3] = rot<T>(y[1][3], s1, c1, sign);
    y[2][1] = rot<T>(y[2][1], h, h, sign);
    y[2][2] = mul_i<T>(y[2][2], sign);
    y[2][3] = rot<T>(y[2][3], -h, h, sign);
    y[3][1] = rot<T>(y[3][1], s1, c1, sign);
    y[3][2] = rot<T>(y[3][2], -h, h, sign);
    y[3][3] = rot<T>(y[3][3], -c1, -s1, sign);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      V2<T> t[4] = {y[0][c], y[1][c], y[2][c], y[3][c]};
      Dft<T, 4>::run(t, sign);
#pragma unroll
      for (int d = 0; d < 4; ++d) v[c + 4 * d] = t[d];
    }
  }
};

// Radix of the next pass for a remaining length rem: 8 while it divides, then
// 4, 2, 3, 5 (any order of the factors gives a correct Stockham FFT); 16 for
// lines of 1024 and more, where it saves a pass (1024 = 16 16 4 instead of
// 8 8 8 2; at shorter lengths the larger in-register DFT measured no faster).
__host__ __device__ constexpr int next_radix(int rem) {
  return (rem >= 1024 && rem % 16 == 0) ? 16
         : (rem % 8 == 0)              ? 8
         : (rem % 4 == 0)              ? 4
         : (rem % 2 == 0)              ? 2
         : (rem % 3 == 0)              ? 3
                                       : 5;
}

// One radix-R pass on NL lines of length N held in LDS, all sizes known at
// compile time.  Layout: interleaved (element q of line c at q*NL + c; the
// strided-axis tiles) or line-major (at c*LSX + q; contiguous lines, LSX >= N).
// Twiddles come from a table tw[k] = exp(-2 pi i k / (N * TWS)).
template <typename T, int R, int N, int NS, int NL, int NT, bool INTERLEAVED, int LSX, int TWS>
__device__ __forceinline__ void ct_pass(V2<T>* buf, const V2<T>* __restrict__ tw, T sign) {
  constexpr int NB = N / R;
  constexpr int TOTAL = NB * NL;
  constexpr int BPT = (TOTAL + NT - 1) / NT;
  constexpr int STEP = (N / (NS * R)) * TWS;
  constexpr int ES = INTERLEAVED ? NL : 1;
  constexpr int LS = INTERLEAVED ? 1 : LSX;
  V2<T> v[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int w = threadIdx.x + b * NT;
    if (TOTAL % NT == 0 || w < TOTAL) {
      const int c = INTERLEAVED ? w % NL : w / NB;
      const int j = INTERLEAVED ? w / NL : w % NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[c * LS + (j + r * NB) * ES];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int w = threadIdx.x + b * NT;
    if (TOTAL % NT == 0 || w < TOTAL) {
      const int c = INTERLEAVED ? w % NL : w / NB;
      const int j = INTERLEAVED ? w / NL : w % NB;
      const int jm = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V2<T> t = tw[r * jm * STEP];
          t.y *= -sign;  // table holds exp(-i...); sign = +1 conjugates
          v[b][r] = mul<T>(v[b][r], t);
        }
      }
      Dft<T, R>::run(v[b], sign);
      const int base = (j / NS) * NS * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[c * LS + (base + r * NS) * ES] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int NS, int NL, int NT, bool INTERLEAVED, int LSX, int TWS>
__device__ __forceinline__ void ct_passes(V2<T>* buf, const V2<T>* __restrict__ tw, T sign) {
  if constexpr (NS < N) {
    constexpr int R = next_radix(N / NS);
    ct_pass<T, R, N, NS, NL, NT, INTERLEAVED, LSX, TWS>(buf, tw, sign);
    ct_passes<T, N, NS * R, NL, NT, INTERLEAVED, LSX, TWS>(buf, tw, sign);
  }
}

// Block-wide copy of COUNT elements (thread t handles e = t + it * NT) in two
// phases: all of a thread's loads first (held in registers), then its stores,
// so every load of the thread is in flight at once.
template <int COUNT, int NT, typename T, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(Load&& load, Store&& store) {
  constexpr int IT = (COUNT + NT - 1) / NT;
  T v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NT;
    if (COUNT % NT == 0 || e < COUNT) v[it] = load(e);
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NT;
    if (COUNT % NT == 0 || e < COUNT) store(e, v[it]);
  }
}

// Full FFT (sign -1 forward, +1 inverse, unnormalised) of NL lines of length N
// in LDS; starts and ends with the block synchronised.
template <typename T, int N, int NL, int NT, bool INTERLEAVED, int LSX, int TWS>
__device__ __forceinline__ void ct_fft(V2<T>* buf, const V2<T>* __restrict__ tw, T sign) {
  ct_passes<T, N, 1, NL, NT, INTERLEAVED, LSX, TWS>(buf, tw, sign);
}

}  // namespace bispec
