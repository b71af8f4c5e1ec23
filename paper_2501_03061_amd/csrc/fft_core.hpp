// Device-side building blocks of the LDS-staged mixed-radix FFT (gfx950).
//
// A 1D transform of compile-time length N is a sequence of Stockham
// autosort stages with radices taken from {2, 3, 4, 5, 6, 8, 9, 10, 12}.  Stage s with radix
// R and span NS (the product of the radices before it) maps butterfly j of a
// line (0 <= j < N/R) as
//     in :  x[j + r*N/R],                          r = 0..R-1
//     tw :  x_r *= w^(r * (j mod NS)),             w = exp(-+ 2 pi i/(NS*R))
//     out:  y[(j/NS)*NS*R + (j mod NS) + r*NS] = DFT_R(x)_r
// so that the result comes out in natural order with no bit reversal.  The
// last stage (NS = N/R) writes positions j + r*N/R, the same set the first
// stage of another transform with the same radix reads, which lets the
// forward and inverse z transforms of the kernel-multiply pass meet in
// registers.
//
// Forward transforms use exp(-i...), inverse exp(+i...), both unnormalised.
// Twiddles come from a table of the N-th roots of unity (FP64 sincospi,
// rounded for FP32), held in LDS; powers w^r are formed by repeated complex
// multiplication.  Composite radices (6, 9, 10, 12) are Cooley-Tukey in
// registers with compile-time twiddles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace px {

template <typename T> struct cpx { T x, y; };

template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // conj(a) * b
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename T> __device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> __device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) {
  if (INV) return {-a.y, a.x};
  return {a.y, -a.x};
}

// ---------------------------------------------------------------- radix kernels
template <typename T, bool INV> __device__ __forceinline__ void dft2(cpx<T>* v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, bool INV> __device__ __forceinline__ void dft3(cpx<T>* v) {
  const T c = T(-0.5);
  const T s = T(0.86602540378443864676372317075294);  // sin(2 pi/3)
  cpx<T> t = cadd(v[1], v[2]);
  cpx<T> d = csub(v[1], v[2]);
  cpx<T> m = {v[0].x + c * t.x, v[0].y + c * t.y};
  // y1 = m -+ i s d, y2 = m +- i s d  (upper sign: forward)
  cpx<T> isd = INV ? cpx<T>{-s * d.y, s * d.x} : cpx<T>{s * d.y, -s * d.x};
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, isd);
  v[2] = csub(m, isd);
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(cpx<T>* v) {
  cpx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  cpx<T> a2 = cadd(v[1], v[3]), a3 = mul_mi<T, INV>(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <typename T, bool INV> __device__ __forceinline__ void dft5(cpx<T>* v) {
  const T c1 = T(0.30901699437494742410229341718282);   // cos(2 pi/5)
  const T c2 = T(-0.80901699437494742410229341718282);  // cos(4 pi/5)
  const T s1 = T(0.95105651629515357211643933337938);   // sin(2 pi/5)
  const T s2 = T(0.58778525229247312916870595463907);   // sin(4 pi/5)
  cpx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  cpx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  cpx<T> a = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
  cpx<T> b = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
  cpx<T> p = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
  cpx<T> q = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
  cpx<T> ip = mul_mi<T, INV>(p), iq = mul_mi<T, INV>(q);  // -i p (fwd) / +i p (inv)
  v[0] = {v[0].x + t1.x + t2.x, v[0].y + t1.y + t2.y};
  v[1] = cadd(a, ip);
  v[4] = csub(a, ip);
  v[2] = cadd(b, iq);
  v[3] = csub(b, iq);
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(cpx<T>* v) {
  const T h = T(0.70710678118654752440084436210485);
  cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  // w8^k for k = 1, 2, 3: fwd (1-i)/sqrt2, -i, (-1-i)/sqrt2; inv conjugates
  cpx<T> o1 = INV ? cpx<T>{h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)}
                  : cpx<T>{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
  cpx<T> o2 = mul_mi<T, INV>(o[2]);
  cpx<T> o3 = INV ? cpx<T>{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)}
                  : cpx<T>{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// Compile-time roots of unity: cos and sin of 2 pi m / R, evaluated by
// constexpr Taylor series after exact reduction of the angle to [-pi/4, pi/4]
// (accurate to about one ulp in double precision).
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_sin_small(double t) {  // |t| <= pi/4
  double term = t, sum = t;
  for (int k = 1; k < 14; ++k) {
    term *= -t * t / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos_small(double t) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -t * t / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// angle 2 pi m / R with exact quadrant reduction on the integer 4 m mod 4 R
constexpr void cx_root(int R, int m, double& c, double& s) {
  m %= R;
  if (m < 0) m += R;
  const long num = 4L * m;             // angle = (num / R) * (pi / 2)
  const long quad = (2 * num + R) / (2 * R);  // nearest multiple of pi/2, 0..4
  const double rem = double(num - quad * R) / double(R) * (kPi / 2.0);  // |rem| <= pi/4
  const double sr = cx_sin_small(rem), cr = cx_cos_small(rem);
  switch (int(quad % 4)) {
    case 0: c = cr; s = sr; break;
    case 1: c = -sr; s = cr; break;
    case 2: c = -cr; s = -sr; break;
    default: c = sr; s = -cr; break;
  }
}

template <int R> struct RootTable {
  double c[R], s[R];
  constexpr RootTable() : c(), s() {
    for (int m = 0; m < R; ++m) cx_root(R, m, c[m], s[m]);
  }
};
template <int R> inline constexpr RootTable<R> kRoots{};

template <typename T, int R, bool INV> __device__ __forceinline__ void dft(cpx<T>* v);

// Composite radix R = A*B (Cooley-Tukey in registers): B-point transforms of
// the A decimated subsequences, twiddles w_R^(a*q), then A-point transforms;
// input index a + A*b, output index q + B*p.
template <typename T, int A, int B, bool INV> __device__ __forceinline__ void dft_ct(cpx<T>* v) {
  constexpr int R = A * B;
  cpx<T> u[A][B];
#pragma unroll
  for (int a = 0; a < A; ++a) {
    cpx<T> s[B];
#pragma unroll
    for (int b = 0; b < B; ++b) s[b] = v[a + A * b];
    dft<T, B, INV>(s);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (a == 0 || q == 0) {
        u[a][q] = s[q];
      } else {
        constexpr const RootTable<R>& tab = kRoots<R>;
        const T c = T(tab.c[(a * q) % R]);
        const T sn = T(INV ? tab.s[(a * q) % R] : -tab.s[(a * q) % R]);
        u[a][q] = {s[q].x * c - s[q].y * sn, s[q].x * sn + s[q].y * c};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < B; ++q) {
    cpx<T> s[A];
#pragma unroll
    for (int a = 0; a < A; ++a) s[a] = u[a][q];
    dft<T, A, INV>(s);
#pragma unroll
    for (int p = 0; p < A; ++p) v[q + B * p] = s[p];
  }
}

// Factor A of a composite length handled by dft_ct<A, R/A>.
template <int R> constexpr int first_factor() {
  return R % 8 == 0 && R > 8 ? 8 : R % 6 == 0 && R > 6 ? 6 : R % 4 == 0 && R > 4 ? 4
       : R % 3 == 0 && R > 3 ? 3 : R % 2 == 0 && R > 2 ? 2 : R % 5 == 0 && R > 5 ? 5 : 1;
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 5) dft5<T, INV>(v);
  else if constexpr (R == 6) dft_ct<T, 2, 3, INV>(v);
  else if constexpr (R == 9) dft_ct<T, 3, 3, INV>(v);
  else if constexpr (R == 10) dft_ct<T, 2, 5, INV>(v);
  else if constexpr (R == 12) dft_ct<T, 4, 3, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else {
    // whole-line transforms (e.g. 72 = 8 x 9) for the register-resident pencils
    constexpr int A = first_factor<R>();
    static_assert(A > 1 && R % A == 0, "length must factor into 2, 3, 5");
    dft_ct<T, A, R / A, INV>(v);
  }
}

// ---------------------------------------------------------------- plans
// Radix sequence per supported length: two stages everywhere, so a 2D
// transform in LDS needs one transposing round trip per axis.  The inverse
// transform uses the reversed sequence so that its first radix equals the
// forward's last.
template <int N> struct Plan;
#define PX_PLAN(N_, NST_, R0_, R1_, R2_) \
  template <> struct Plan<N_> { static constexpr int nst = NST_; static constexpr int rad[3] = {R0_, R1_, R2_}; };
PX_PLAN(16, 2, 4, 4, 1)
PX_PLAN(24, 2, 8, 3, 1)
PX_PLAN(32, 2, 8, 4, 1)
PX_PLAN(40, 2, 8, 5, 1)
PX_PLAN(48, 2, 8, 6, 1)
PX_PLAN(60, 2, 6, 10, 1)
PX_PLAN(64, 2, 8, 8, 1)
PX_PLAN(72, 2, 8, 9, 1)
PX_PLAN(80, 2, 8, 10, 1)
PX_PLAN(90, 2, 9, 10, 1)
PX_PLAN(96, 2, 8, 12, 1)
PX_PLAN(120, 2, 10, 12, 1)
#undef PX_PLAN

// Radix and span of stage S of the plan's radix sequence (INV = false) or of
// the reversed sequence (INV = true; the inverse transforms use it, and so
// does the forward x transform of the pair product, see pass 1).
template <int N, int S, bool INV> struct StageOf {
  static constexpr int nst = Plan<N>::nst;
  static constexpr int idx = INV ? (nst - 1 - S) : S;
  static constexpr int R = Plan<N>::rad[idx];
  static constexpr int NS = [] {
    int p = 1;
    for (int s = 0; s < S; ++s) p *= Plan<N>::rad[INV ? (Plan<N>::nst - 1 - s) : s];
    return p;
  }();
};

// ---------------------------------------------------------------- line geometry
// A set of NL lines of length N in LDS; element e of line l sits at
// l*LS + e*ES.  LINE_FAST selects which index varies fastest across
// consecutive butterflies (threads): the line (for strided lines, so that
// neighbouring threads touch neighbouring addresses) or the position in the
// line (for contiguous lines).
template <int N, int NL, int LS, int ES, bool LINE_FAST> struct Lines {
  static constexpr int n = N, nl = NL, ls = LS, es = ES;
  static constexpr bool line_fast = LINE_FAST;
};

template <class G, int R> __device__ __forceinline__ void decode(int b, int& line, int& j) {
  if constexpr (G::line_fast) {
    line = b % G::nl;
    j = b / G::nl;
  } else {
    j = b % (G::n / R);
    line = b / (G::n / R);
  }
}

template <int N, int R> constexpr int butterflies_per_thread(int nl, int nt) {
  return (nl * (N / R) + nt - 1) / nt;
}

// Twiddle w^(r*k) for r = 1..R-1 applied in place; k = j mod NS, base root
// index k*(N/(NS*R)) in the N-entry table (forward table; inverse conjugates).
// FP32: every power is read from the table (each correctly rounded from FP64),
// so the transform carries no error growth from repeated products (measured:
// the same speed, a 4x smaller FP32 energy error at 96^3).  FP64: powers by
// repeated multiplication (error r * 1e-16, far below tolerance).
template <typename T, int N, int R, int NS, bool INV>
__device__ __forceinline__ void twiddle(cpx<T>* v, int j, const cpx<T>* tw) {
  if constexpr (NS == 1) return;
  const int k = j % NS;
  constexpr int STEP = N / (NS * R);
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cpx<T> w = tw[r * k * STEP];
      if (INV) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
  } else {
    cpx<T> w = tw[k * STEP];
    if (INV) w.y = -w.y;
    cpx<T> wr = w;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = cmul(v[r], wr);
      if (r + 1 < R) wr = cmul(wr, w);
    }
  }
}

// Output position (within its line) of element r of butterfly j.
template <int R, int NS> __device__ __forceinline__ int out_pos(int j, int r) {
  return (j / NS) * NS * R + (j % NS) + r * NS;
}

// One LDS -> LDS Stockham stage over all lines of geometry G, in place: every
// thread loads its butterflies into registers, the block synchronises, then
// each butterfly is transformed and written back.  Ends with a barrier.
template <typename T, class G, int R, int NS, bool INV, int NT>
__device__ __forceinline__ void stage_lds(cpx<T>* lds, const cpx<T>* tw) {
  constexpr int NB = G::nl * (G::n / R);
  constexpr int BPT = (NB + NT - 1) / NT;
  cpx<T> v[BPT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      int line, j;
      decode<G, R>(b, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = lds[line * G::ls + (j + r * (G::n / R)) * G::es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      int line, j;
      decode<G, R>(b, line, j);
      twiddle<T, G::n, R, NS, INV>(v[k], j, tw);
      dft<T, R, INV>(v[k]);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[line * G::ls + out_pos<R, NS>(j, r) * G::es] = v[k][r];
    }
  }
  __syncthreads();
}

// One out-of-place Stockham stage, src -> dst (both LDS, same geometry).  No
// barrier inside: the caller separates stages that depend on each other.
template <typename T, class G, int R, int NS, bool INV, int NT>
__device__ __forceinline__ void stage_pp(const cpx<T>* src, cpx<T>* dst, const cpx<T>* tw) {
  constexpr int NB = G::nl * (G::n / R);
  constexpr int BPT = (NB + NT - 1) / NT;
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = threadIdx.x + k * NT;
    if (NB % NT == 0 || b < NB) {
      int line, j;
      decode<G, R>(b, line, j);
      cpx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[line * G::ls + (j + r * (G::n / R)) * G::es];
      twiddle<T, G::n, R, NS, INV>(v, j, tw);
      dft<T, R, INV>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[line * G::ls + out_pos<R, NS>(j, r) * G::es] = v[r];
    }
  }
}

// Run stages [S0, S1) of the length-N transform over geometry G, LDS -> LDS,
// in the forward (REV = false) or reversed radix order.
template <typename T, class G, bool INV, int NT, int S, int S1, bool REV = INV>
__device__ __forceinline__ void stages_lds(cpx<T>* lds, const cpx<T>* tw) {
  if constexpr (S < S1) {
    using St = StageOf<G::n, S, REV>;
    stage_lds<T, G, St::R, St::NS, INV, NT>(lds, tw);
    stages_lds<T, G, INV, NT, S + 1, S1, REV>(lds, tw);
  }
}

}  // namespace px
