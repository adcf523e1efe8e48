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
// registers, the work group synchronises, then all threads store.
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

// Radix schedule of one line length, passed by value to kernels.
struct FftSched {
  int n;       // line length
  int npass;
  int r[12];   // radices, applied in order
  int tw_stride;  // table index step: table holds exp(-2 pi i k / Nt), Nt = n * tw_stride
};

// Lines in LDS: element q of line c sits at buf[c * ls + q * es].  With
// interleaved = true, consecutive threads walk lines first (good when es == 1
// is false, i.e. lines are interleaved); otherwise butterflies first.
template <typename T, int R, int E, int NT>
__device__ __forceinline__ void stockham_pass(V2<T>* buf, int n, int ns, int nl, int es, int ls, bool interleaved,
                                              const V2<T>* __restrict__ tw, int tw_stride, T sign) {
  constexpr int BPT = (E + R - 1) / R;
  const int nb = n / R;
  const int total = nb * nl;
  const int step = (n / (ns * R)) * tw_stride;
  V2<T> v[BPT][R];
  int jj[BPT], cc[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int w = threadIdx.x + b * NT;
    int j, c;
    if (interleaved) { c = w % nl; j = w / nl; } else { j = w % nb; c = w / nb; }
    jj[b] = j;
    cc[b] = c;
    if (w < total) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[c * ls + (j + r * nb) * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int w = threadIdx.x + b * NT;
    if (w < total) {
      const int j = jj[b], c = cc[b];
      const int jm = j % ns;
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V2<T> t = tw[r * jm * step];
          t.y *= -sign;  // table is exp(-i...); sign = -1 keeps it, +1 conjugates
          v[b][r] = mul<T>(v[b][r], t);
        }
      }
      Dft<T, R>::run(v[b], sign);
      const int base = (j / ns) * ns * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[c * ls + (base + r * ns) * es] = v[b][r];
    }
  }
  __syncthreads();
}

// Full FFT of nl lines of length s.n in LDS.  sign = -1 forward, +1 inverse
// (unnormalised).  Requires s.n * nl <= NT * E.  Ends with a barrier.
template <typename T, int E, int NT>
__device__ void lds_fft(V2<T>* buf, const FftSched& s, int nl, int es, int ls, bool interleaved,
                        const V2<T>* __restrict__ tw, T sign) {
  int ns = 1;
  for (int p = 0; p < s.npass; ++p) {
    const int R = s.r[p];
    switch (R) {
      case 8: stockham_pass<T, 8, E, NT>(buf, s.n, ns, nl, es, ls, interleaved, tw, s.tw_stride, sign); break;
      case 4: stockham_pass<T, 4, E, NT>(buf, s.n, ns, nl, es, ls, interleaved, tw, s.tw_stride, sign); break;
      case 2: stockham_pass<T, 2, E, NT>(buf, s.n, ns, nl, es, ls, interleaved, tw, s.tw_stride, sign); break;
      case 3: stockham_pass<T, 3, E, NT>(buf, s.n, ns, nl, es, ls, interleaved, tw, s.tw_stride, sign); break;
      case 5: stockham_pass<T, 5, E, NT>(buf, s.n, ns, nl, es, ls, interleaved, tw, s.tw_stride, sign); break;
      default: break;
    }
    ns *= R;
  }
}

}  // namespace bispec
