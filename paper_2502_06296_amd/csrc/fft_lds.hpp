// In-LDS complex FFT engine for the x and y real transforms.
//
// A workgroup holds LPW complex lines of compile-time length N in LDS. Two
// real lines are carried as the real and imaginary parts of one complex
// line, so every real transform of the solver runs as a complex transform
// followed by the split into two packed real spectra (paper App. A layout).
// The transform is a Stockham autosort over radix-16/9/8/5/4/3/2 passes: each
// pass reads R elements spaced N/R apart, applies the twiddles and an
// R-point DFT in registers, and writes them back R-interleaved; every pass is
// separated from the next by a workgroup barrier, and TPL threads share a
// line.
#pragma once
#include <hip/hip_runtime.h>

namespace pf {

template <typename T> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename T>
__device__ __forceinline__ cplx<T> mkc(T x, T y) { cplx<T> r; r.x = x; r.y = y; return r; }
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mkc<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mkc<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mkc<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mkc<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> rot90(cplx<T> a) {
  return INV ? mkc<T>(-a.y, a.x) : mkc<T>(a.y, -a.x);
}

// LDS index with one pad element per 16, to spread the R-strided writes of
// the early passes over the banks.
__device__ __forceinline__ constexpr int lds_idx(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_len(int n) { return n + (n >> 4) + 1; }

// ------------------------------------------------------------ small DFTs
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cplx<T> &a, cplx<T> &b) {
  cplx<T> t = a;
  a = cadd<T>(t, b);
  b = csub<T>(t, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cplx<T> &v0, cplx<T> &v1, cplx<T> &v2, cplx<T> &v3) {
  cplx<T> t0 = cadd<T>(v0, v2), t1 = csub<T>(v0, v2);
  cplx<T> t2 = cadd<T>(v1, v3), t3 = rot90<T, INV>(csub<T>(v1, v3));
  v0 = cadd<T>(t0, t2);
  v2 = csub<T>(t0, t2);
  v1 = cadd<T>(t1, t3);
  v3 = csub<T>(t1, t3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(cplx<T> &v0, cplx<T> &v1, cplx<T> &v2) {
  const T h = T(0.5);
  const T s = INV ? T(0.86602540378443864676372317075294) : T(-0.86602540378443864676372317075294);
  cplx<T> t = cadd<T>(v1, v2);
  cplx<T> d = csub<T>(v1, v2);
  cplx<T> m = mkc<T>(v0.x - h * t.x, v0.y - h * t.y);
  cplx<T> u = mkc<T>(-s * d.y, s * d.x);   // i*s*(v1 - v2)
  v0 = cadd<T>(v0, t);
  v1 = cadd<T>(m, u);
  v2 = csub<T>(m, u);
}

// 5-point DFT from the sums and differences of the mirrored inputs:
// X_k = x0 + cos(2 pi k/5)-weighted sums -+ i sin(2 pi k/5)-weighted
// differences, with X_{5-k} the same terms with the other sign of i.
template <typename T, bool INV>
__device__ __forceinline__ void dft5(cplx<T> &v0, cplx<T> &v1, cplx<T> &v2, cplx<T> &v3, cplx<T> &v4) {
  const T c1 = T(0.30901699437494742410229341718282);   // cos(2 pi / 5)
  const T c2 = T(-0.80901699437494742410229341718282);  // cos(4 pi / 5)
  const T s1 = T(0.95105651629515357211643933337938);   // sin(2 pi / 5)
  const T s2 = T(0.58778525229247312916870595463907);   // sin(4 pi / 5)
  const cplx<T> t1 = cadd<T>(v1, v4), t2 = cadd<T>(v2, v3);
  const cplx<T> t3 = csub<T>(v1, v4), t4 = csub<T>(v2, v3);
  const cplx<T> a1 = mkc<T>(v0.x + c1 * t1.x + c2 * t2.x, v0.y + c1 * t1.y + c2 * t2.y);
  const cplx<T> a2 = mkc<T>(v0.x + c2 * t1.x + c1 * t2.x, v0.y + c2 * t1.y + c1 * t2.y);
  // -i b (forward) or +i b (inverse) of the sine-weighted differences
  const cplx<T> b1 = rot90<T, INV>(mkc<T>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  const cplx<T> b2 = rot90<T, INV>(mkc<T>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  v0 = cadd<T>(v0, cadd<T>(t1, t2));
  v1 = cadd<T>(a1, b1);
  v4 = csub<T>(a1, b1);
  v2 = cadd<T>(a2, b2);
  v3 = csub<T>(a2, b2);
}

// 8-point DFT in natural order, as two 4-point DFTs of the even and odd
// samples joined by the eighth roots of unity.
template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T> *v) {
  const T r = T(0.70710678118654752440084436210485);
  cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  // o_k * w^k, w = exp(-+ 2 pi i / 8)
  cplx<T> w1 = INV ? mkc<T>(r * (o1.x - o1.y), r * (o1.x + o1.y))
                   : mkc<T>(r * (o1.x + o1.y), r * (o1.y - o1.x));
  cplx<T> w2 = rot90<T, INV>(o2);
  cplx<T> w3 = INV ? mkc<T>(-r * (o3.x + o3.y), r * (o3.x - o3.y))
                   : mkc<T>(r * (o3.y - o3.x), -r * (o3.x + o3.y));
  v[0] = cadd<T>(e0, o0); v[4] = csub<T>(e0, o0);
  v[1] = cadd<T>(e1, w1); v[5] = csub<T>(e1, w1);
  v[2] = cadd<T>(e2, w2); v[6] = csub<T>(e2, w2);
  v[3] = cadd<T>(e3, w3); v[7] = csub<T>(e3, w3);
}

// 16-point DFT as 4 x 4: DFTs over n1 for each n2, twiddle by w16^(n2 k1),
// DFTs over n2 for each k1; output index k1 + 4 k2.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cplx<T> *v) {
  const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
  const T c2 = T(0.70710678118654752440084436210485);
  for (int n2 = 0; n2 < 4; ++n2) dft4<T, INV>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
  // after this v[n2 + 4*k1] holds Y_{n2}[k1]
  const T sg = INV ? T(1) : T(-1);
  // twiddles w16^(n2*k1) for n2, k1 in 1..3: exponents 1,2,3,2,4,6,3,6,9
  auto tw = [&](cplx<T> a, T c, T s) { return mkc<T>(a.x * c - a.y * (sg * s), a.x * (sg * s) + a.y * c); };
  v[1 + 4] = tw(v[1 + 4], c1, s1);
  v[1 + 8] = tw(v[1 + 8], c2, c2);
  v[1 + 12] = tw(v[1 + 12], s1, c1);
  v[2 + 4] = tw(v[2 + 4], c2, c2);
  v[2 + 8] = rot90<T, INV>(v[2 + 8]);
  v[2 + 12] = tw(v[2 + 12], -c2, c2);
  v[3 + 4] = tw(v[3 + 4], s1, c1);
  v[3 + 8] = tw(v[3 + 8], -c2, c2);
  v[3 + 12] = tw(v[3 + 12], -c1, -s1);
  cplx<T> o[16];
  for (int k1 = 0; k1 < 4; ++k1) {
    cplx<T> a = v[4 * k1 + 0], b = v[4 * k1 + 1], c = v[4 * k1 + 2], d = v[4 * k1 + 3];
    dft4<T, INV>(a, b, c, d);
    o[k1] = a; o[k1 + 4] = b; o[k1 + 8] = c; o[k1 + 12] = d;
  }
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

// 9-point DFT as 3 x 3: DFTs over n1 for each n2, twiddle by w9^(n2 k1),
// DFTs over n2 for each k1; output index k1 + 3 k2.
template <typename T, bool INV>
__device__ __forceinline__ void dft9(cplx<T> *v) {
  const T c1 = T(0.76604444311897803520239265055542);   // cos(2 pi / 9)
  const T s1 = T(0.64278760968653932632264340990726);   // sin(2 pi / 9)
  const T c2 = T(0.17364817766693034885171662676931);   // cos(4 pi / 9)
  const T s2 = T(0.98480775301220805936674302458952);   // sin(4 pi / 9)
  const T c4 = T(-0.93969262078590838405410927732473);  // cos(8 pi / 9)
  const T s4 = T(0.34202014332566873304409961468226);   // sin(8 pi / 9)
  for (int n2 = 0; n2 < 3; ++n2) dft3<T, INV>(v[n2], v[n2 + 3], v[n2 + 6]);
  // after this v[n2 + 3*k1] holds Y_{n2}[k1]; twiddle exponents n2*k1 = 1, 2, 2, 4
  const T sg = INV ? T(1) : T(-1);
  auto tw = [&](cplx<T> a, T c, T s) { return mkc<T>(a.x * c - a.y * (sg * s), a.x * (sg * s) + a.y * c); };
  v[1 + 3] = tw(v[1 + 3], c1, s1);
  v[1 + 6] = tw(v[1 + 6], c2, s2);
  v[2 + 3] = tw(v[2 + 3], c2, s2);
  v[2 + 6] = tw(v[2 + 6], c4, s4);
  cplx<T> o[9];
  for (int k1 = 0; k1 < 3; ++k1) {
    cplx<T> a = v[3 * k1 + 0], b = v[3 * k1 + 1], c = v[3 * k1 + 2];
    dft3<T, INV>(a, b, c);
    o[k1] = a; o[k1 + 3] = b; o[k1 + 6] = c;
  }
  for (int i = 0; i < 9; ++i) v[i] = o[i];
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_r(cplx<T> *v) {
  if constexpr (R == 2) dft2<T, INV>(v[0], v[1]);
  else if constexpr (R == 3) dft3<T, INV>(v[0], v[1], v[2]);
  else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 5) dft5<T, INV>(v[0], v[1], v[2], v[3], v[4]);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 9) dft9<T, INV>(v);
  else if constexpr (R == 16) dft16<T, INV>(v);
}

// radix of the next pass for the remaining length REM; radix order RO = 1
// caps the radix at 8 (more passes, fewer values per thread)
template <int REM, int RO = 0>
__host__ __device__ constexpr int pick_radix() {
  return (RO == 0 && REM % 16 == 0 && REM != 32) ? 16
         : (REM % 8 == 0)             ? 8
         : (REM % 4 == 0)             ? 4
         : (REM % 2 == 0)             ? 2
         : (REM % 9 == 0)             ? 9
         : (REM % 3 == 0)             ? 3
         : (REM % 5 == 0)             ? 5
                                      : 0;
}

// Twiddles w[r] = W^(e r), r = 1..R-1, of one butterfly from at most two
// table reads: W^e and, for R >= 8, W^(4e); the others are products of
// these, at most four multiplications deep (a few ulp), instead of R-1
// table reads per butterfly.
template <typename T, int R>
__device__ __forceinline__ void pass_twiddles(cplx<T> (&w)[R], const cplx<T> *__restrict__ tw, int e) {
  w[1] = tw[e];
  if constexpr (R >= 3) w[2] = cmul<T>(w[1], w[1]);
  if constexpr (R >= 4) w[3] = cmul<T>(w[2], w[1]);
  if constexpr (R == 5) w[4] = cmul<T>(w[2], w[2]);
  if constexpr (R >= 8) {
    w[4] = tw[4 * e];
#pragma unroll
    for (int r = 5; r < 8; ++r) w[r] = cmul<T>(w[4], w[r - 4]);
  }
  if constexpr (R == 9) w[8] = cmul<T>(w[4], w[4]);
  if constexpr (R >= 16) {
    w[8] = cmul<T>(w[4], w[4]);
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul<T>(w[8], w[r - 8]);
  }
}

// One Stockham pass of radix R on a line of N: every thread reads the R
// inputs j + r N/R of its butterflies through src, applies the twiddles and
// the R-point DFT in registers, and writes the outputs through dst (Stockham
// autosort order). LDS_IN / LDS_OUT tell whether src / dst are the LDS line:
// a pass that reads and writes it in place separates its reads from its
// writes by a barrier, and every pass that writes it ends with one. A first
// pass may read straight from global memory and a last pass may write
// straight to it, which saves a sweep over the LDS line and two barriers.
// tw[t] = exp(-2 pi i t / N).
template <typename T, int N, int R, int NS, int TPL, bool INV, bool LDS_IN, bool LDS_OUT, class Src,
          class Dst>
__device__ __forceinline__ void stockham_pass_io(const cplx<T> *__restrict__ tw, int t, Src src,
                                                 Dst dst) {
  constexpr int NB = N / R;
  constexpr int IT = (NB + TPL - 1) / TPL;
  cplx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = t + it * TPL;
    if (NB % TPL == 0 || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = src(j + r * NB);
      if constexpr (NS > 1) {
        cplx<T> w[R];
        pass_twiddles<T, R>(w, tw, (j % NS) * (N / (NS * R)));
#pragma unroll
        for (int r = 1; r < R; ++r) v[it][r] = INV ? cmulc<T>(v[it][r], w[r]) : cmul<T>(v[it][r], w[r]);
      }
      dft_r<T, R, INV>(v[it]);
    }
  }
  if constexpr (LDS_IN && LDS_OUT) __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = t + it * TPL;
    if (NB % TPL == 0 || j < NB) {
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) dst(base + r * NS, v[it][r]);
    }
  }
  if constexpr (LDS_OUT) __syncthreads();
}

// GIN: the first pass reads the line through src instead of LDS (nothing
// may be reading the LDS line when the transform starts); GOUT: the last
// pass writes the result through dst instead of LDS (the LDS line is left
// partly stale). Otherwise the line must be in LDS, published by a barrier,
// and the result is left there, published by a barrier.
template <typename T, int N, int NS, int TPL, bool INV, bool GIN, bool GOUT, int RO, class Src, class Dst>
__device__ __forceinline__ void fft_passes_io(cplx<T> *buf, const cplx<T> *__restrict__ tw, int t,
                                              Src src, Dst dst) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix<N / NS, RO>();
    static_assert(R != 0, "transform length must be 2^a 3^b 5^c");
    constexpr bool gin = GIN && NS == 1, gout = GOUT && NS * R == N;
    auto lrd = [buf](int i) { return buf[lds_idx(i)]; };
    auto lwr = [buf](int i, const cplx<T> &x) { buf[lds_idx(i)] = x; };
    if constexpr (gin && gout) stockham_pass_io<T, N, R, NS, TPL, INV, false, false>(tw, t, src, dst);
    else if constexpr (gin) stockham_pass_io<T, N, R, NS, TPL, INV, false, true>(tw, t, src, lwr);
    else if constexpr (gout) stockham_pass_io<T, N, R, NS, TPL, INV, true, false>(tw, t, lrd, dst);
    else stockham_pass_io<T, N, R, NS, TPL, INV, true, true>(tw, t, lrd, lwr);
    fft_passes_io<T, N, NS * R, TPL, INV, GIN, GOUT, RO>(buf, tw, t, src, dst);
  }
}

template <typename T, int N, int TPL, bool INV, bool GIN, bool GOUT, int RO = 0, class Src, class Dst>
__device__ __forceinline__ void fft_line_io(cplx<T> *buf, const cplx<T> *__restrict__ tw, int t,
                                            Src src, Dst dst) {
  fft_passes_io<T, N, 1, TPL, INV, GIN, GOUT, RO>(buf, tw, t, src, dst);
}

// The first pass of fft_line_io split in two, so that a line's inputs can
// be loaded while the previous line is being transformed: first_load reads
// the values the thread's first-pass butterflies take (radix R of the first
// pass, no twiddles) into registers; fft_from_regs transforms them, writes
// the first pass's output to the LDS line (ending with a barrier), and
// fft_rest runs the remaining passes as fft_line_io does.
template <int N, int TPL, int RO>
struct FirstPass {
  static constexpr int R = pick_radix<N, RO>();
  static constexpr int NB = N / R;
  static constexpr int IT = (NB + TPL - 1) / TPL;
  static_assert(R != 0 && R < N, "a first pass of a longer transform");
};
template <int N, int TPL, int RO, class V, int IT, int R, class Src>
__device__ __forceinline__ void first_load(V (&v)[IT][R], int t, Src src) {
  using F = FirstPass<N, TPL, RO>;
  static_assert(IT == F::IT && R == F::R, "registers of the first pass");
#pragma unroll
  for (int it = 0; it < F::IT; ++it) {
    const int j = t + it * TPL;
    if (F::NB % TPL == 0 || j < F::NB) {
#pragma unroll
      for (int r = 0; r < F::R; ++r) v[it][r] = src(j + r * F::NB);
    }
  }
}
template <typename T, int N, int TPL, bool INV, int RO, class V, int IT, int R>
__device__ __forceinline__ void fft_from_regs(cplx<T> *buf, const V (&in)[IT][R], int t) {
  using F = FirstPass<N, TPL, RO>;
  static_assert(IT == F::IT && R == F::R, "registers of the first pass");
  cplx<T> v[F::IT][F::R];
#pragma unroll
  for (int it = 0; it < F::IT; ++it) {
    const int j = t + it * TPL;
    if (F::NB % TPL == 0 || j < F::NB) {
#pragma unroll
      for (int r = 0; r < F::R; ++r) v[it][r] = mkc<T>((T)in[it][r].x, (T)in[it][r].y);
      dft_r<T, F::R, INV>(v[it]);
#pragma unroll
      for (int r = 0; r < F::R; ++r) buf[lds_idx(j * F::R + r)] = v[it][r];
    }
  }
  __syncthreads();
}
template <typename T, int N, int TPL, bool INV, bool GOUT, int RO, class Dst>
__device__ __forceinline__ void fft_rest(cplx<T> *buf, const cplx<T> *__restrict__ tw, int t, Dst dst) {
  fft_passes_io<T, N, FirstPass<N, TPL, RO>::R, TPL, INV, false, GOUT, RO>(
      buf, tw, t, [](int) { return cplx<T>{}; }, dst);
}

// Full complex transform of one LDS line, in place (unnormalised). Every
// thread of the workgroup must call it (it contains barriers).
template <typename T, int N, int TPL, bool INV>
__device__ __forceinline__ void fft_line(cplx<T> *buf, const cplx<T> *__restrict__ tw, int t) {
  auto none_rd = [](int) { return cplx<T>{}; };
  auto none_wr = [](int, const cplx<T> &) {};
  fft_line_io<T, N, TPL, INV, false, false>(buf, tw, t, none_rd, none_wr);
}

// Split the transform Z of z = a + i b (a, b real) into the spectra of a and
// b at mode q (1 <= q < N/2):
//   A_q = (Z_q + conj Z_{N-q}) / 2,  B_q = (Z_q - conj Z_{N-q}) / (2i).
template <typename T>
__device__ __forceinline__ void split_pair(cplx<T> zq, cplx<T> zn, cplx<T> &A, cplx<T> &B) {
  const T h = T(0.5);
  A = mkc<T>(h * (zq.x + zn.x), h * (zq.y - zn.y));
  B = mkc<T>(h * (zq.y + zn.y), h * (zn.x - zq.x));
}

// Inverse of split_pair: from the half spectra A_q, B_q (1 <= q < N/2)
// rebuild Z_q = A_q + i B_q and Z_{N-q} = conj(A_q) + i conj(B_q).
template <typename T>
__device__ __forceinline__ void join_pair(cplx<T> A, cplx<T> B, cplx<T> &zq, cplx<T> &zn) {
  zq = mkc<T>(A.x - B.y, A.y + B.x);
  zn = mkc<T>(A.x + B.y, B.x - A.y);
}

}  // namespace pf
