// HIP kernels of libshot for gfx950 (MI355X).
//
// The heat apply K v = F^{-1}(h (.) F v) (Sec. 3.2) is split at its two global
// dependency points into
//   * row kernels: one workgroup per pair of mirror latitude rows (j, nlat-1-j).
//     The two real rows ride in one complex FFT (real part row j, imaginary part
//     row j'), done in LDS by a mixed-radix Stockham FFT; the result is folded
//     into the equatorially even/odd combinations E_m = F_m(j) + F_m(j') and
//     O_m = F_m(j) - F_m(j') that the folded Legendre stage consumes.  The
//     Sinkhorn pointwise update of Alg. 1 is fused between the inverse FFT of
//     one heat apply and the forward FFT of the next one, so a field never
//     makes an extra trip through HBM.
//   * Legendre kernels: one workgroup per order m (and chunk of items):
//     analysis f_lm = sum_j a_j P̄_l^m(x_j) {E|O}_m(j), multiply by h_l, and
//     synthesis G_m(j) = sum_l b_lm P̄_l^m(x_j), all for the same m, so the
//     spectral coefficients never leave the workgroup.  P̄_l^m comes from a
//     table streamed from HBM or from the float64 three-term recurrence.
// Folding uses P̄_l^m(-x) = (-1)^{l+m} P̄_l^m(x): only rows j <= nlat/2 are
// touched by the Legendre stage.
//
// Spectral workspace layout per item: [m][j][parity] complex, m < L,
// j < h = ceil(nlat/2), parity 0 = E (even l-m), 1 = O (odd l-m).
// Reductions are per-workgroup float64 partial sums written to fixed slots and
// summed later in a fixed order, so results are deterministic (no float atomics).

#include <cfloat>
#include <climits>

#include <hip/hip_ext.h>

#include "host_math.h"
#include "shot_internal.h"

namespace shot {

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by s*i (s = +-1)
template <typename T>
__device__ __forceinline__ cpx<T> cmul_si(cpx<T> a, T s) { return {-s * a.y, s * a.x}; }

// ---------------------------------------------------------------------------
// Mixed-radix Stockham FFT in LDS, radices 2, 3, 4, 5.  sign = -1 forward,
// +1 inverse (unnormalised).  All threads of the block must call it.  Returns
// the buffer that holds the result (natural order).
// ---------------------------------------------------------------------------
// cos and sin of 2 pi e / R, e = 0 .. R-1: the internal twiddles of the
// register-level composite radices
template <int R>
struct UnitRoots;
template <>
struct UnitRoots<8> {
  static constexpr double c[8] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440,
                                  -1.0, -0.70710678118654752440, 0.0, 0.70710678118654752440};
  static constexpr double s[8] = {0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440,
                                  0.0, -0.70710678118654752440, -1.0, -0.70710678118654752440};
};
template <>
struct UnitRoots<9> {
  static constexpr double c[9] = {1.0, 0.76604444311897803520, 0.17364817766693034885, -0.5,
                                  -0.93969262078590838405, -0.93969262078590838405, -0.5,
                                  0.17364817766693034885, 0.76604444311897803520};
  static constexpr double s[9] = {0.0, 0.64278760968653932632, 0.98480775301220805937, 0.86602540378443864676,
                                  0.34202014332566873304, -0.34202014332566873304, -0.86602540378443864676,
                                  -0.98480775301220805937, -0.64278760968653932632};
};

template <typename T, int R>
__device__ __forceinline__ void butterfly(cpx<T>* v, T s) {
  if constexpr (R == 2) {
    cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    cpx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    cpx<T> t2 = cadd(v[1], v[3]), t3 = cmul_si(csub(v[1], v[3]), s);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else if constexpr (R == 3) {
    const T c = (T)-0.5, sn = s * (T)0.86602540378443864676;
    cpx<T> t = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    cpx<T> base = {v[0].x + c * t.x, v[0].y + c * t.y};
    cpx<T> rot = cmul_si(d, sn);  // i * sn * d
    v[0] = cadd(v[0], t);
    v[1] = cadd(base, rot);
    v[2] = csub(base, rot);
  } else if constexpr (R == 5) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = s * (T)0.95105651629515357212, s2 = s * (T)0.58778525229247312917;
    cpx<T> t1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
    cpx<T> t2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
    cpx<T> b1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    cpx<T> b2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    cpx<T> e1 = {s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
    cpx<T> e2 = {s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
    cpx<T> r1 = cmul_si(e1, (T)1), r2 = cmul_si(e2, (T)1);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(b1, r1);
    v[4] = csub(b1, r1);
    v[2] = cadd(b2, r2);
    v[3] = csub(b2, r2);
  } else if constexpr (R == 8 || R == 9) {
    // R = R1 R2 in registers: with r = R2 r1 + r2 and q = q1 + R1 q2,
    // X[q] = sum_r2 w_R2^(r2 q2) w_R^(r2 q1) sum_r1 w_R1^(r1 q1) v[R2 r1 + r2]
    constexpr int R1 = R == 9 ? 3 : 4, R2 = R / R1;
    cpx<T> y[R2][R1];
#pragma unroll
    for (int r2 = 0; r2 < R2; ++r2) {
#pragma unroll
      for (int r1 = 0; r1 < R1; ++r1) y[r2][r1] = v[R2 * r1 + r2];
      butterfly<T, R1>(y[r2], s);
    }
#pragma unroll
    for (int r2 = 1; r2 < R2; ++r2)
#pragma unroll
      for (int q1 = 1; q1 < R1; ++q1) {
        const int e = r2 * q1;  // w_R^e = cos(2 pi e / R) + i s sin(2 pi e / R)
        y[r2][q1] = cmul(y[r2][q1], cpx<T>{(T)UnitRoots<R>::c[e], s * (T)UnitRoots<R>::s[e]});
      }
#pragma unroll
    for (int q1 = 0; q1 < R1; ++q1) {
      cpx<T> z[R2];
#pragma unroll
      for (int r2 = 0; r2 < R2; ++r2) z[r2] = y[r2][q1];
      butterfly<T, R2>(z, s);
#pragma unroll
      for (int q2 = 0; q2 < R2; ++q2) v[q1 + R1 * q2] = z[q2];
    }
  }
}

template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                               int N, int Ns, int nb, const cpx<T>* __restrict__ tw, T sign) {
  // nb independent transforms of length N stored back to back
  const int NR = N / R;
  const int twstride = N / (Ns * R);
  for (int bb = threadIdx.x; bb < nb * NR; bb += blockDim.x) {
    const int t = bb / NR, b = bb - t * NR;
    const cpx<T>* s = src + t * N;
    cpx<T>* d = dst + t * N;
    const int k = b % Ns;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[b + r * NR];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cpx<T> w = tw[r * k * twstride];
      w.y *= -sign;  // table holds exp(-2 pi i k/N); inverse uses the conjugate
      v[r] = cmul(v[r], w);
    }
    butterfly<T, R>(v, sign);
    const int base = (b / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[base + r * Ns] = v[r];
  }
}

// Stockham stage of any radix R (the primes above 5 of ring lengths that are
// not 2,3,5-smooth): each thread forms whole outputs, output q of butterfly b
// being sum_r src[b + r N/R] w^{r (k N/(Ns R) + q N/R)} with w the length-N
// root, so every term costs one table lookup.
template <typename T>
__device__ __forceinline__ void stockham_stage_generic(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst, int N, int Ns,
                                       int R, int nb, const cpx<T>* __restrict__ tw, T sign) {
  const int NR = N / R;
  const int twstride = N / (Ns * R);
  for (int o = threadIdx.x; o < nb * N; o += blockDim.x) {
    const int t = o / N, rem = o - t * N;
    const int q = rem / NR, b = rem - q * NR;
    const int k = b % Ns;
    const cpx<T>* s = src + t * N;
    const int e = k * twstride + q * NR;
    cpx<T> acc = {(T)0, (T)0};
    int idx = 0;  // r * e mod N, advanced by e (< N, so one subtraction wraps it)
    int r = 0;
    // eight terms per step: their LDS reads are all in flight before the first use
    for (; r + 8 <= R; r += 8) {
      int ix[8];
      cpx<T> v[8], w[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        ix[j] = idx;
        idx += e;
        idx = idx >= N ? idx - N : idx;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        v[j] = s[b + (r + j) * NR];
        w[j] = tw[ix[j]];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        w[j].y *= -sign;  // table holds exp(-2 pi i k/N); inverse uses the conjugate
        acc = cadd(acc, cmul(v[j], w[j]));
      }
    }
    for (; r < R; ++r) {
      cpx<T> w = tw[idx];
      w.y *= -sign;
      acc = cadd(acc, cmul(s[b + r * NR], w));
      idx += e;
      idx = idx >= N ? idx - N : idx;
    }
    dst[t * N + (b / Ns) * Ns * R + k + q * Ns] = acc;
  }
}

template <typename T>
__device__ __forceinline__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, int N, int nb, const int* fac, int nfac,
                           const cpx<T>* __restrict__ tw, T sign) {
  int Ns = 1;
  cpx<T>* src = a;
  cpx<T>* dst = b;
  for (int s = 0; s < nfac; ++s) {
    const int R = fac[s];
    switch (R) {
      case 2: stockham_stage<T, 2>(src, dst, N, Ns, nb, tw, sign); break;
      case 3: stockham_stage<T, 3>(src, dst, N, Ns, nb, tw, sign); break;
      case 4: stockham_stage<T, 4>(src, dst, N, Ns, nb, tw, sign); break;
      case 5: stockham_stage<T, 5>(src, dst, N, Ns, nb, tw, sign); break;
      default: stockham_stage_generic<T>(src, dst, N, Ns, R, nb, tw, sign); break;
    }
    __syncthreads();
    cpx<T>* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
}

// Compile-time factorisation (same radix order as the host: 4, 2, 3, 5) for
// the common transform lengths: every stage's length, stride and twiddle step
// become constants, so the index arithmetic needs no runtime division.
struct FacList {
  int n;
  int r[12];
};
__host__ __device__ constexpr FacList factorize(int N) {
  FacList f{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  const int rs[4] = {4, 2, 3, 5};
  for (int i = 0; i < 4; ++i)
    while (N % rs[i] == 0 && f.n < 12) {
      f.r[f.n++] = rs[i];
      N /= rs[i];
    }
  return f;
}
// The compile-time stages fuse a radix 4 with the radix 2 and pairs of
// radix 3 into register-level radix-8 and radix-9 stages: fewer LDS passes
// and barriers, and every stage of a 1440-point row fits one pass of 512
// threads (4, 8, 9, 5 instead of 4, 4, 2, 3, 3, 5; three heavier stages
// 16, 10, 9 leave too few threads busy and measured slower).
__host__ __device__ constexpr FacList fuse_factors(FacList f) {
  FacList g{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  int n4 = 0, n2 = 0, n3 = 0, n5 = 0;
  for (int i = 0; i < f.n; ++i) {
    if (f.r[i] == 4) ++n4;
    else if (f.r[i] == 2) ++n2;
    else if (f.r[i] == 3) ++n3;
    else ++n5;
  }
  const int n8 = (n4 > 0 && n2 > 0) ? 1 : 0;
  for (int i = 0; i < n4 - n8; ++i) g.r[g.n++] = 4;
  for (int i = 0; i < n8; ++i) g.r[g.n++] = 8;
  for (int i = 0; i < n2 - n8; ++i) g.r[g.n++] = 2;
  for (int i = 0; i < n3 / 2; ++i) g.r[g.n++] = 9;
  for (int i = 0; i < n3 % 2; ++i) g.r[g.n++] = 3;
  for (int i = 0; i < n5; ++i) g.r[g.n++] = 5;
  return g;
}
__host__ __device__ constexpr int fac_prefix(FacList f, int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= f.r[i];
  return p;
}

template <typename T, int R, int N, int Ns, int NB>
__device__ __forceinline__ void stockham_stage_c(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                                 const cpx<T>* __restrict__ tw, T sign) {
  constexpr int NR = N / R;
  constexpr int twstride = N / (Ns * R);
  for (int bb = threadIdx.x; bb < NB * NR; bb += blockDim.x) {
    const int t = bb / NR, b = bb - t * NR;
    const cpx<T>* s = src + t * N;
    cpx<T>* d = dst + t * N;
    const int k = b % Ns;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[b + r * NR];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cpx<T> w = tw[r * k * twstride];
      w.y *= -sign;
      v[r] = cmul(v[r], w);
    }
    butterfly<T, R>(v, sign);
    const int base = (b / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[base + r * Ns] = v[r];
  }
}

template <typename T, int N, int NB, int S>
__device__ __forceinline__ void fft_stages_c(cpx<T>*& src, cpx<T>*& dst, const cpx<T>* tw, T sign) {
  constexpr FacList F = fuse_factors(factorize(N));
  if constexpr (S < F.n) {
    constexpr int R = F.r[S];
    constexpr int Ns = fac_prefix(F, S);
    stockham_stage_c<T, R, N, Ns, NB>(src, dst, tw, sign);
    __syncthreads();
    cpx<T>* t = src;
    src = dst;
    dst = t;
    fft_stages_c<T, N, NB, S + 1>(src, dst, tw, sign);
  }
}

// Length chosen at compile time (NC > 0) or at run time (NC == 0).
template <typename T, int NC, int NB>
__device__ __forceinline__ cpx<T>* fft_any(cpx<T>* a, cpx<T>* b, int N, const int* fac, int nfac,
                                           const cpx<T>* tw, T sign) {
  if constexpr (NC > 0) {
    cpx<T>* src = a;
    cpx<T>* dst = b;
    fft_stages_c<T, NC, NB, 0>(src, dst, tw, sign);
    return src;
  } else {
    return fft_lds<T>(a, b, N, NB, fac, nfac, tw, sign);
  }
}

// ---------------------------------------------------------------------------
// Cross-lane exchanges without LDS round trips: DPP row permutes for lane
// bits 0-3, permlane swaps (gfx950) for bits 4 and 5.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dpp_f(float v, int ctrl_sel) {
  int x = __float_as_int(v);
  int r;
  switch (ctrl_sel) {
    case 0: r = __builtin_amdgcn_update_dpp(0, x, 0x140, 0xf, 0xf, false); break;  // row_mirror (bit 3)
    case 1: r = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, false); break;  // row_half_mirror (bit 2)
    case 2: r = __builtin_amdgcn_update_dpp(0, x, 0x4e, 0xf, 0xf, false); break;   // quad_perm [2,3,0,1] (bit 1)
    default: r = __builtin_amdgcn_update_dpp(0, x, 0xb1, 0xf, 0xf, false); break;  // quad_perm [1,0,3,2] (bit 0)
  }
  return __int_as_float(r);
}

__device__ __forceinline__ double dpp_d(double v, int ctrl_sel) {
  const unsigned long long u = __double_as_longlong(v);
  float lo = __int_as_float((int)(u & 0xffffffffull)), hi = __int_as_float((int)(u >> 32));
  const unsigned long long rl = (unsigned)__float_as_int(dpp_f(lo, ctrl_sel));
  const unsigned long long rh = (unsigned)__float_as_int(dpp_f(hi, ctrl_sel));
  return __longlong_as_double((long long)(rl | (rh << 32)));
}

// new value = X(lane) + X(lane ^ 32) for lanes < 32, Y(lane ^ 32) + Y(lane) above.
__device__ __forceinline__ float swap_add32(float X, float Y) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(X), __float_as_uint(Y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_add16(float X, float Y) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(X), __float_as_uint(Y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double swap_add32(double X, double Y) {
  const unsigned long long x = __double_as_longlong(X), y = __double_as_longlong(Y);
  auto lo = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
  auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
  const double a = __longlong_as_double((long long)((unsigned long long)lo[0] | ((unsigned long long)hi[0] << 32)));
  const double b = __longlong_as_double((long long)((unsigned long long)lo[1] | ((unsigned long long)hi[1] << 32)));
  return a + b;
}
__device__ __forceinline__ double swap_add16(double X, double Y) {
  const unsigned long long x = __double_as_longlong(X), y = __double_as_longlong(Y);
  auto lo = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
  auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
  const double a = __longlong_as_double((long long)((unsigned long long)lo[0] | ((unsigned long long)hi[0] << 32)));
  const double b = __longlong_as_double((long long)((unsigned long long)lo[1] | ((unsigned long long)hi[1] << 32)));
  return a + b;
}

// v of the lane and of its partner across lane bit 4 (permlane16) or bit 5
// (permlane32), returned as (value of the lower lane, value of the upper lane)
// so that both partners see the same ordered pair.
__device__ __forceinline__ void lane_pair16(double v, double& lo, double& hi) {
  const unsigned long long x = __double_as_longlong(v);
  auto a = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
  auto b = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(x >> 32), false, false);
  lo = __longlong_as_double((long long)((unsigned long long)a[0] | ((unsigned long long)b[0] << 32)));
  hi = __longlong_as_double((long long)((unsigned long long)a[1] | ((unsigned long long)b[1] << 32)));
}
__device__ __forceinline__ void lane_pair32(double v, double& lo, double& hi) {
  const unsigned long long x = __double_as_longlong(v);
  auto a = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
  auto b = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(x >> 32), false, false);
  lo = __longlong_as_double((long long)((unsigned long long)a[0] | ((unsigned long long)b[0] << 32)));
  hi = __longlong_as_double((long long)((unsigned long long)a[1] | ((unsigned long long)b[1] << 32)));
}

// Wave-wide all-reduction with a commutative op (sum, min, max): at every
// step a lane and its partner combine the same two values, so all 64 lanes
// end with the identical, run-to-run deterministic result.
template <typename Op>
__device__ __forceinline__ double wave_allreduce(double v, Op op) {
  v = op(v, dpp_d(v, 3));  // lane ^ 1
  v = op(v, dpp_d(v, 2));  // lane ^ 2
  v = op(v, dpp_d(v, 1));  // mirror within 8 lanes
  v = op(v, dpp_d(v, 0));  // mirror within 16 lanes
  double lo, hi;
  lane_pair16(v, lo, hi);
  v = op(lo, hi);
  lane_pair32(v, lo, hi);
  return op(lo, hi);
}
struct OpAdd {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMin {
  __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct OpMax {
  __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
__device__ __forceinline__ double wave_sum(double v) { return wave_allreduce(v, OpAdd()); }
__device__ __forceinline__ double wave_min(double v) { return wave_allreduce(v, OpMin()); }
__device__ __forceinline__ double wave_max(double v) { return wave_allreduce(v, OpMax()); }

// ---------------------------------------------------------------------------
// Deterministic block reduction: every thread receives the same value (the
// wave partials are combined in wave order by each thread).
// ---------------------------------------------------------------------------

__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  return r;
}

// Sums of r[0] and r[3], minimum of r[1], maximum of r[2] over the block,
// combined in wave order (as block_sum) with one pair of barriers; sh holds
// 4 doubles per wave.
__device__ void block_reduce4(double* r, double* sh) {
  r[0] = wave_sum(r[0]);
  r[1] = wave_min(r[1]);
  r[2] = wave_max(r[2]);
  r[3] = wave_sum(r[3]);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0)
    for (int i = 0; i < 4; ++i) sh[4 * w + i] = r[i];
  __syncthreads();
  double a = 0.0, b = INFINITY, c = -INFINITY, d = 0.0;
  for (int i = 0; i < nw; ++i) {
    a += sh[4 * i];
    b = fmin(b, sh[4 * i + 1]);
    c = fmax(c, sh[4 * i + 2]);
    d += sh[4 * i + 3];
  }
  r[0] = a;
  r[1] = b;
  r[2] = c;
  r[3] = d;
}

__device__ double block_min(double v, double* sh) {
  v = wave_min(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < nw; ++i) r = fmin(r, sh[i]);
  return r;
}

__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < nw; ++i) r = fmax(r, sh[i]);
  return r;
}

// Non-finite outputs count as -inf so that the ratio of that half is -inf.
template <typename T>
__device__ __forceinline__ void track_minmax(double& mn, double& mx, T v) {
  const double d = isfinite(v) ? (double)v : -INFINITY;
  mn = fmin(mn, d);
  mx = fmax(mx, d);
}

template <typename T>
__device__ __forceinline__ bool bad_kernel_value(T x) {
  return !(x > (T)0) || !isfinite(x);
}

// Term u^(-eps/tau) of the unbalanced gauge sums (Alg. 1), taken in the field
// precision: a float32 scaling gives a float32 power (about one ulp, as the
// scaling itself carries); a float64 power of it cost more than the rest of
// an unbalanced row launch.  The sums themselves stay float64.
template <typename T>
__device__ __forceinline__ double gauge_term(T u, double eot) {
  return (double)pow(u, (T)(-eot));
}

// The unbalanced update x -> x^lam (lam = tau/(tau+eps)) and the new value's
// gauge-sum term x^(-lam eps/tau), both from one base-2 logarithm in float32:
// exp2(lam log2 x) is within about |log2 x| ulp of the correctly rounded power
// (about 1e-6 relative for scalings within 2^+-16), and the term's exponent is
// damped by eps/tau.  Zero, infinite and negative x give what the powers give.
// float64 fields keep the library powers.
template <typename T>
__device__ __forceinline__ T unbalanced_update(T x, double lam, double eot, double& term) {
  if constexpr (sizeof(T) == 4) {
    const float y = (float)lam * log2f(x);
    term = (double)exp2f(-(float)eot * y);
    return exp2f(y);
  } else {
    const T xn = pow(x, (T)lam);
    term = gauge_term(xn, eot);
    return xn;
  }
}

template <typename T>
__device__ __forceinline__ T* ubuf_of(const RowArgs<T>& A, int k) { return (k & 1) ? A.ubuf1 : A.ubuf0; }
template <typename T>
__device__ __forceinline__ T* vbuf_of(const RowArgs<T>& A, int k) { return (k & 1) ? A.vbuf1 : A.vbuf0; }

// Gauge g_k: after iteration k the Alg. 1 scalings are u_k = u_hat/g_k and
// v_k = g_k v_hat, with g_k = s = sum u_hat (balanced) or exp(-c/eps) with
// c = tau/2 (log sum a p u_hat^(-eps/tau) - log sum a q v_hat^(-eps/tau)).
template <typename T>
__device__ double gauge(const RowArgs<T>& A, const ItemDev& I, int it, int k, double* sh) {
  const double* R = A.red + ((size_t)(k & 1) * A.nitems_all + it) * (size_t)A.hs * RED_SLOTS;
  double s0 = 0.0, s1 = 0.0;
  for (int q = threadIdx.x; q < A.h; q += blockDim.x) {
    s0 += R[(size_t)q * RED_SLOTS + 0];
    s1 += R[(size_t)q * RED_SLOTS + 1];
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  if (I.balanced) return s0;
  const double c = 0.5 * I.tau * (log(s0) - log(s1));
  return exp(-c / I.eps);
}

// Folded spectrum entry (E, O) of order m and row pair jp of item `it`: read
// from the spectrum, or, for an order that the preceding Legendre launch cut
// into parts, the sum of the parts' partial sums taken in part order.
template <typename T>
__device__ __forceinline__ void load_spec_pair(const RowArgs<T>& A, const cpx<T>* spec, int it, int m, int jp,
                                               cpx<T>& ge, cpx<T>& go) {
  if (A.cut) {
    const int2 c = A.cut[m];
    if (c.x > 1) {
      const int rel = it - A.item0, chunk = rel / A.cut_ib, i = rel - chunk * A.cut_ib;
      const cpx<T>* pb = static_cast<const cpx<T>*>(A.pbuf) + (size_t)chunk * A.npb * A.cut_ib * 2 * A.h +
                         (size_t)i * 2 * A.h + 2 * jp;
      ge = {(T)0, (T)0};
      go = {(T)0, (T)0};
      for (int p = 0; p < c.x; ++p) {
        const cpx<T>* q = pb + (size_t)(c.y + p) * A.cut_ib * 2 * A.h;
        ge = cadd(ge, q[0]);
        go = cadd(go, q[1]);
      }
      return;
    }
  }
  const cpx<T>* sp = spec + ((size_t)m * A.h + jp) * 2;
  ge = sp[0];
  go = sp[1];
}

// Bijection of [0, h): workgroup b runs on XCD b % 8; XCD x gets the
// contiguous row-pair range starting at x*(h/8) + min(x, h%8).
__device__ __forceinline__ int xcd_row_pair(int b, int h) {
  const int q = h >> 3, r = h & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Adjoint notes (balanced Alg. 1, reverse mode).  Forward iteration k:
//   A = K v_{k-1}, u-hat = p / A, B = K u-hat, v-hat = q / B, s = sum u-hat,
//   u_k = u-hat / s, v_k = s v-hat;  cost R = sum a (eps log u_T p + eps log v_T q).
// Only v_k feeds the next iteration, so the reverse sweep carries v-bar:
//   s-bar = sum v-bar (.) v-hat  (- sum u-bar_T (.) u-hat / s^2 at k = T)
//   q-bar += s v-bar v-hat / q,  B-bar = -s v-bar v-hat^2 / q
//   u-hat-bar = s-bar + K^T B-bar (+ u-bar_T / s at k = T)
//   p-bar += u-hat-bar u-hat / p,  A-bar = -u-hat-bar u-hat^2 / p,  v-bar_{k-1} = K^T A-bar
// with K^T x = a (.) K(x / a): the forward FFT skips the area weights and the
// inverse side multiplies by them.  u-bar_T = eps a p / u_T, v-bar_T = eps a q / v_T,
// and the cost contributes eps a log u_T to p-bar and eps a log v_T to q-bar.
//
// Unbalanced iteration k (lambda = tau/(tau+eps), eta = eps/tau):
//   u-hat = (p / K v_{k-1})^lambda, v-hat = (q / K u-hat)^lambda,
//   S_A = sum a p u-hat^-eta, S_B = sum a q v-hat^-eta, g = (S_A / S_B)^(-1/(2 eta)),
//   u_k = u-hat / g, v_k = g v-hat;  cost R = tau sum a (p (1 - u_T^-eta) + q (1 - v_T^-eta)).
// K v_{k-1} = p u-hat^(-1/lambda) and K u-hat = q v-hat^(-1/lambda) are recovered
// pointwise.  Reverse step k, given v-bar_k (at k = T: eps a q v_T^(-eta-1), and
// u-bar_T = eps a p u_T^(-eta-1)):
//   g-bar = sum v-bar v-hat (- sum u-bar_T u-hat / g^2 at k = T)
//   S_A-bar = -g-bar g / (2 eta S_A),  S_B-bar = g-bar g / (2 eta S_B)
//   v-hat-bar = g v-bar - eta S_B-bar a q v-hat^(-eta-1)
//   q-bar += S_B-bar a v-hat^-eta + lambda v-hat-bar v-hat / q,  B-bar = -lambda v-hat-bar v-hat^(1+1/lambda) / q
//   u-hat-bar = K^T B-bar - eta S_A-bar a p u-hat^(-eta-1) (+ u-bar_T / g at k = T)
//   p-bar += S_A-bar a u-hat^-eta + lambda u-hat-bar u-hat / p,  A-bar = -lambda u-hat-bar u-hat^(1+1/lambda) / p
//   v-bar_{k-1} = K^T A-bar;  the cost adds tau a (1 - u_T^-eta) to p-bar and tau a (1 - v_T^-eta) to q-bar.

// Kernel ratio of one half-iteration (min over all rows of K. / max), folded
// into the item's running minimum.  Called by one block per item.
template <typename T>
__device__ void kratio_fold(const RowArgs<T>& A, int it, int k, int slot, double* sh) {
  const double* R = A.red + ((size_t)(k & 1) * A.nitems_all + it) * (size_t)A.hs * RED_SLOTS;
  double mn = INFINITY, mx = -INFINITY;
  for (int q = threadIdx.x; q < A.h; q += blockDim.x) {
    mn = fmin(mn, R[(size_t)q * RED_SLOTS + slot]);
    mx = fmax(mx, R[(size_t)q * RED_SLOTS + slot + 1]);
  }
  mn = block_min(mn, sh);
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) {
    const double r = (mx > 0.0 && isfinite(mn)) ? mn / mx : -INFINITY;
    A.kr[it] = fmin(A.kr[it], r);
  }
}

// ---------------------------------------------------------------------------
// Row kernel.  grid = (ceil(h / RPW) groups of RPW row pairs, items), block 256.
// Each row pair (j, nlat-1-j) rides in one complex FFT; the RPW pairs of a
// group share the twiddles and the barriers of the staged FFTs, and their
// spectral entries (m, j..j+RPW-1) are contiguous in memory.  Per-row-pair
// partial sums are written at the group's first pair (the other slots of the
// group get the neutral element) so all consumers still reduce over j < h.
// ---------------------------------------------------------------------------
// Transform of one ring pair's packed row (length n = RG->len), in LDS
// buffers a and b of at least max(n, RG->bm) entries; returns the buffer
// holding the result in its first n entries.  Lengths with a prime factor
// above 64 use Bluestein's identity nk = (n^2 + k^2 - (k - n)^2) / 2: with
// c_j = exp(sign i pi j^2 / n), X_k = c_k sum_j (x_j c_j) conj(c_{k-j}), a
// cyclic convolution of length bm evaluated with two power-of-two FFTs and
// the plan's spectrum of the conjugate chirp (the inverse direction uses the
// complex conjugates of both tables).  tw: twiddles of the FFT length used.
template <typename T>
__device__ __forceinline__ cpx<T>* ring_fft(cpx<T>* a, cpx<T>* b, int n, const RingDev* RG, const cpx<T>* tw,
                                            const cpx<T>* __restrict__ blu, T sign) {
  // one inlined FFT, run once (direct) or twice (the convolution's forward
  // and inverse transforms): each inlined copy carries every radix stage
  const int M = RG->bm;
  const bool bs = M > 0;
  const cpx<T>* ch = blu + RG->ch_off;
  const cpx<T>* bh = blu + RG->bh_off;
  const bool conj = sign > (T)0;
  if (bs) {
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
      cpx<T> c = j < n ? ch[j] : cpx<T>{(T)0, (T)0};
      if (conj) c.y = -c.y;
      a[j] = j < n ? cmul(a[j], c) : cpx<T>{(T)0, (T)0};
    }
    __syncthreads();
  }
  cpx<T>* y = a;
  for (int pass = 0; pass < (bs ? 2 : 1); ++pass) {
    const T sg = bs ? (pass ? (T)1 : (T)-1) : sign;
    y = fft_lds<T>(y, y == a ? b : a, bs ? M : n, 1, bs ? RG->bm_fac : RG->fac, bs ? RG->bm_nfac : RG->nfac, tw,
                   sg);
    if (bs && pass == 0) {
      for (int k = threadIdx.x; k < M; k += blockDim.x) {
        cpx<T> f = bh[k];
        if (conj) f.y = -f.y;
        y[k] = cmul(y[k], f);
      }
      __syncthreads();
    }
  }
  if (bs) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      cpx<T> c = ch[k];
      if (conj) c.y = -c.y;
      y[k] = cmul(y[k], c);
    }
    __syncthreads();
  }
  return y;
}

// a[e][r] for e, r in {0, 1} by selects (a run-time index would put the
// array in scratch memory)
template <typename T>
__device__ __forceinline__ T pick2(const T (&a)[2][2], int e, int r) {
  const T x = r ? a[0][1] : a[0][0], y = r ? a[1][1] : a[1][0];
  return e ? y : x;
}

template <typename T, int RPW, int NC, int BS = 256>
__global__ void __launch_bounds__(BS) row_kernel(RowArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = A.L, h = A.h;
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous range of groups so that neighbouring rows' spectral entries
  // (adjacent in memory) meet in the same L2.
  const int ngroups = (h + RPW - 1) / RPW;
  const int jp0 = (A.rpair ? A.rpair[blockIdx.x] : xcd_row_pair(blockIdx.x, ngroups)) * RPW;
  // HEALPix: this pair's rings (one pair per group), else uniform rows
  const RingDev* RG = A.ring ? A.ring + jp0 : nullptr;
  const int N = RG ? RG->len : (NC > 0 ? NC : A.nlon);
  const int NB = RG ? A.nbuf : N;  // LDS stride: the longest ring or Bluestein convolution
  cpx<T>* buf0 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* buf1 = buf0 + RPW * NB;
  cpx<T>* twl = buf1 + RPW * NB;
  __shared__ double sh[16];
  __shared__ int sh_bad;
  __shared__ T awl[RPW];

  const int np = min(RPW, h - jp0);  // active pairs of this group
  const int it = A.item0 + blockIdx.y;
  const ItemDev I = A.items[it];
  const int nlat = A.nlat;
  const int tid = threadIdx.x, bs = blockDim.x;
  cpx<T>* spec = A.spec + I.soff;  // [m][j][E/O]
  const int mode = A.mode;
  // the marginals, as global pointers (from the descriptor in memory the
  // compiler could not tell, and flat loads also count as LDS operations)
  using GT = const __attribute__((address_space(1))) T;
  GT* P = (GT*)static_cast<const T*>(I.p);
  GT* Q = (GT*)static_cast<const T*>(I.q);
  if (tid < RPW) awl[tid] = (tid < np) ? A.aw[jp0 + tid] : (T)0;
  if (tid == 0) sh_bad = 0;

  double g = 1.0;
  if (mode == ROW_FINAL) g = gauge(A, I, it, A.k, sh);
  else if (mode == ROW_SINK_U && A.gk) g = A.gk[it];
  else if (mode == ROW_SINK_U && A.k > 1) g = gauge(A, I, it, A.k - 1, sh);
  __syncthreads();

// per-element pair geometry: pr = pair in group, c = column
#define ROW_PAIR_SETUP(idx)                                                        \
  const int pr = (idx) / N, c = (idx) - pr * N;                                    \
  const int jp = jp0 + pr;                                                         \
  const int j2 = nlat - 1 - jp;                                                    \
  const bool eq = (jp == j2);                                                      \
  const long long r1 = I.foff + (RG ? (long long)RG->off1 : (long long)jp * N);    \
  const long long r2 = I.foff + (RG ? (long long)RG->off2 : (long long)j2 * N);    \
  const T aj = awl[pr];

  if (mode == ROW_FINAL) {
    const T* uh = ubuf_of(A, A.k) + I.foff;
    const T* vh = vbuf_of(A, A.k) + I.foff;
    const double lg = log(g);
    double acc = 0.0;
    for (int idx = tid; idx < np * N; idx += bs) {
      ROW_PAIR_SETUP(idx)
      for (int rr = 0; rr < (eq ? 1 : 2); ++rr) {
        const long long fidx = (rr ? r2 : r1) + c;
        const long long fi = fidx - I.foff;
        const double phi = I.eps * (log((double)uh[fi]) - lg);
        const double psi = I.eps * (log((double)vh[fi]) + lg);
        if (A.out) A.out[fidx] = (T)phi;
        if (A.out2) A.out2[fidx] = (T)psi;
        const double pv = P[fidx], qv = Q[fidx];
        if (I.balanced) acc += (double)aj * (phi * pv + psi * qv);
        else acc += (double)aj * (I.tau * (1.0 - exp(-phi / I.tau)) * pv +
                                  I.tau * (1.0 - exp(-psi / I.tau)) * qv);
      }
    }
    acc = block_sum(acc, sh);
    if (tid < np) A.prep[((size_t)it * A.hs + jp0 + tid) * 4 + 3] = (tid == 0) ? acc : 0.0;
    if (A.kr && blockIdx.x == 0 && A.k >= 1) kratio_fold(A, it, A.k, 4, sh);
    return;
  }

  // twiddles of the row length, or of the convolution length of a Bluestein ring
  const cpx<T>* twsrc = RG ? A.ring_tw + (RG->bm ? RG->bm_twoff : RG->twoff) : A.tw;
  const int ntw = (RG && RG->bm) ? RG->bm : N;
  // staged in LDS (always: a pointer that could point to LDS or to global
  // memory would turn every twiddle read of the FFT stages into a flat load)
  for (int i = tid; i < ntw; i += bs) twl[i] = twsrc[i];
  const cpx<T>* tws = twl;
  cpx<T>* X = buf0;
  const bool has_inverse = (mode == ROW_INV || mode == ROW_SINK_U || mode == ROW_SINK_V || mode == ROW_CHECK ||
                            mode == ROW_ADJ_A || mode == ROW_ADJ_VB || mode == ROW_ADJU_A ||
                            (mode == ROW_ADJU_V1 && A.k < A.kT));
  // Sinkhorn halves: the marginal (and, on check iterations, the previous u)
  // at this thread's columns are loaded now, at in-bounds addresses, so that
  // their latency hides behind the inverse FFT (up to PF columns per thread)
  constexpr int PF = 2;
  const bool sink = (mode == ROW_SINK_U || mode == ROW_SINK_V || mode == ROW_CHECK);
  const bool pre = sink && np * N <= PF * bs;
  const bool chk_u = (mode == ROW_SINK_U || mode == ROW_CHECK) && A.chk_slot >= 0;
  T pfv[PF][2], pfu[PF][2];
  if (pre) {
    GT* Fm = mode == ROW_SINK_V ? Q : P;
    const T* uo = ubuf_of(A, A.k - 1);
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int idx = min(tid + e * bs, np * N - 1);
      ROW_PAIR_SETUP(idx)
      (void)eq;
      (void)aj;
      pfv[e][0] = Fm[r1 + c];
      pfv[e][1] = Fm[r2 + c];
      pfu[e][0] = pfu[e][1] = (T)0;
      if (chk_u) {
        pfu[e][0] = uo[r1 + c];
        pfu[e][1] = uo[r2 + c];
      }
    }
  }
  if (has_inverse && RG) {
    // HEALPix ring pair: row r's field is sum_{|m| < L} G_m e^{i m (phi0 + 2 pi k/N)}
    // with G_{-m} = conj(G_m); with P_m = G_m e^{i m phi0}, order m lands in bin
    // m mod N and -m in bin -m mod N of the pair's packed spectrum
    // Z = C_j + i C_j' (orders beyond the ring's length alias, as the samples do).
    // Short rings collect many orders per bin: G threads share a bin (orders
    // split by stride G N) and their partials are added in a fixed order.
    __shared__ cpx<T> ringpart[BS];
    const cpx<T>* ph = A.ring_ph + (size_t)jp0 * L;
    const bool eq = (jp0 == nlat - 1 - jp0);
    const int G = N >= bs ? 1 : bs / N;  // N * G <= bs = BS
    for (int t = tid; t < N * G; t += bs) {
      const int c = t % N, g = t / N;
      cpx<T> z = {(T)0, (T)0};
      for (int m = c + g * N; m < L; m += G * N) {
        cpx<T> ge, go;
        load_spec_pair(A, spec, it, m, jp0, ge, go);
        const cpx<T> a = cmul(cadd(ge, go), ph[m]);
        const cpx<T> b = eq ? cpx<T>{(T)0, (T)0} : cmul(csub(ge, go), ph[m]);
        z.x += a.x - b.y;
        z.y += a.y + b.x;
      }
      for (int m = (c == 0 ? N : N - c) + g * N; m < L; m += G * N) {
        cpx<T> ge, go;
        load_spec_pair(A, spec, it, m, jp0, ge, go);
        const cpx<T> a = cmul(cadd(ge, go), ph[m]);
        const cpx<T> b = eq ? cpx<T>{(T)0, (T)0} : cmul(csub(ge, go), ph[m]);
        z.x += a.x + b.y;
        z.y += -a.y + b.x;
      }
      if (G == 1) buf0[c] = z;
      else ringpart[t] = z;
    }
    if (G > 1) {
      __syncthreads();
      for (int c = tid; c < N; c += bs) {
        cpx<T> z = ringpart[c];
        for (int g = 1; g < G; ++g) z = cadd(z, ringpart[g * N + c]);
        buf0[c] = z;
      }
    }
    __syncthreads();
    X = ring_fft<T>(buf0, buf1, N, RG, tws, A.ring_blu, (T)1);
  } else if (has_inverse) {
    // G_j[m] = GE + GO, G_j'[m] = GE - GO; Z[m] = G_j[m] + i G_j'[m] and its
    // Hermitian mirror Z[N-m] = conj(G_j[m]) + i conj(G_j'[m]); zero elsewhere.
    for (int idx = tid; idx < RPW * (N - 2 * L + 1); idx += bs) {
      const int pr = idx / (N - 2 * L + 1), c = L + idx % (N - 2 * L + 1);
      buf0[pr * N + c] = {(T)0, (T)0};
    }
    for (int idx = tid; idx < RPW * L; idx += bs) {
      const int m = idx / RPW, pr = idx - m * RPW;
      const int jp = jp0 + pr;
      cpx<T> ge = {(T)0, (T)0}, go = {(T)0, (T)0};
      if (pr < np) load_spec_pair(A, spec, it, m, jp, ge, go);
      const bool eq = (jp == nlat - 1 - jp);
      const cpx<T> a = cadd(ge, go);
      const cpx<T> b = eq ? cpx<T>{(T)0, (T)0} : csub(ge, go);
      buf0[pr * N + m] = {a.x - b.y, a.y + b.x};                       // a + i b
      if (m > 0) buf0[pr * N + N - m] = {a.x + b.y, -a.y + b.x};       // conj(a) + i conj(b)
    }
    __syncthreads();
    X = fft_any<T, NC, RPW>(buf0, buf1, N, A.fac, A.nfac, tws, (T)1);
  } else {
    __syncthreads();
  }

  if (mode == ROW_INV) {
    for (int idx = tid; idx < np * N; idx += bs) {
      ROW_PAIR_SETUP(idx)
      const T s = A.wts_out ? aj : (T)1;
      const cpx<T> z = X[pr * N + c];
      A.out[r1 + c] = z.x * s;
      if (!eq) A.out[r2 + c] = z.y * s;
    }
    return;
  }

  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  double kmin = INFINITY, kmax = -INFINITY;  // raw heat-kernel outputs of this group
  bool bad = false;
  if (mode == ROW_SINK_U || mode == ROW_CHECK) {
    // u_hat_k = f(p / (g_{k-1} K v_hat_{k-1})); residual of iteration k-1:
    // u_{k-1} (.) K v_{k-1} - p = u_hat_{k-1} (.) K v_hat_{k-1} - p.
    const T gs = (T)g;
    const T* uo = ubuf_of(A, A.k - 1) + I.foff;
    T* un = ubuf_of(A, A.k) + I.foff;
    const bool chk = (A.chk_slot >= 0);
    for (int idx = tid, e = 0; idx < np * N; idx += bs, ++e) {
      ROW_PAIR_SETUP(idx)
      const cpx<T> z = X[pr * N + c];
      T nv[2];
      for (int rr = 0; rr < (eq ? 1 : 2); ++rr) {
        const long long fidx = (rr ? r2 : r1) + c;
        const long long fi = fidx - I.foff;
        const T kraw = rr ? z.y : z.x;
        const T pv = pre ? pick2(pfv, e, rr) : P[fidx];
        if (chk) {
          const double r = (double)(pre ? pick2(pfu, e, rr) : uo[fi]) * (double)kraw - (double)pv;
          acc2 += r * r;
        }
        if (mode == ROW_CHECK) { nv[rr] = (T)0; continue; }
        const T kv = gs * kraw;
        bad |= bad_kernel_value(kv);
        track_minmax(kmin, kmax, kraw);
        T u = pv / kv;
        double gt = 0.0;
        if (!I.balanced) u = unbalanced_update(u, I.lam, I.eot, gt);
        if (A.store_field) un[fi] = u;
        nv[rr] = u;
        acc0 += I.balanced ? (double)u : (double)aj * (double)pv * gt;
      }
      if (mode == ROW_SINK_U) X[pr * N + c] = {nv[0], eq ? (T)0 : nv[1]};
    }
  } else if (mode == ROW_SINK_V) {
    // v_hat_k = f(q / K u_hat_k): Alg. 1 updates v from u before the gauge step.
    T* vn = vbuf_of(A, A.k) + I.foff;
    for (int idx = tid, e = 0; idx < np * N; idx += bs, ++e) {
      ROW_PAIR_SETUP(idx)
      const cpx<T> z = X[pr * N + c];
      T nv[2];
      for (int rr = 0; rr < (eq ? 1 : 2); ++rr) {
        const long long fidx = (rr ? r2 : r1) + c;
        const T kraw = rr ? z.y : z.x;
        bad |= bad_kernel_value(kraw);
        track_minmax(kmin, kmax, kraw);
        const T qv = pre ? pick2(pfv, e, rr) : Q[fidx];
        T v = qv / kraw;
        if (!I.balanced) {
          double gt;
          v = unbalanced_update(v, I.lam, I.eot, gt);
          acc1 += (double)aj * (double)qv * gt;
        }
        if (A.store_field) vn[fidx - I.foff] = v;
        nv[rr] = v;
      }
      X[pr * N + c] = {nv[0], eq ? (T)0 : nv[1]};
    }
  } else if (mode == ROW_ADJ_START || mode == ROW_ADJ_A || mode == ROW_ADJ_VB) {
    // Reverse sweep of the balanced iteration (see adjoint notes above).
    const double s = A.gk[it];
    const T ss = (T)s;
    const T* uh = ubuf_of(A, 0) + I.foff;  // u-hat of the iteration being reversed
    const T* vh = vbuf_of(A, 0) + I.foff;  // v-hat (of k for START, of k-1 for VB)
    const T ea = (T)I.eps;
    T sbar = (T)0;
    if (mode == ROW_ADJ_A) {
      double sb = 0.0;
      for (int q = tid; q < h; q += bs) sb += A.adjp[(size_t)it * A.hs + q];
      sbar = (T)block_sum(sb, sh);
    }
    for (int idx = tid; idx < np * N; idx += bs) {
      ROW_PAIR_SETUP(idx)
      const cpx<T> z = (mode == ROW_ADJ_START) ? cpx<T>{(T)0, (T)0} : X[pr * N + c];
      T nv[2];
      for (int rr = 0; rr < (eq ? 1 : 2); ++rr) {
        const long long fidx = (rr ? r2 : r1) + c;
        const long long fi = fidx - I.foff;
        const T kt = aj * (rr ? z.y : z.x);  // K^T applied: a (.) (synthesised field)
        if (mode == ROW_ADJ_A) {
          const T u = uh[fi], pv = P[fidx];
          T ub = sbar + kt;
          if (A.k == A.kT) ub += ea * aj * pv / u;  // u-bar_T / s_T = eps a p / u-hat_T
          A.gA[fidx] += ub * u / pv;
          nv[rr] = -ub * u * u / pv;
        } else {
          const T v = vh[fi], qv = Q[fidx];
          T vb;
          if (mode == ROW_ADJ_START) {
            const T u = uh[fi], pv = P[fidx];
            const T uT = u / ss, vT = ss * v;
            A.gA[fidx] = ea * aj * log(uT);  // direct terms of the cost
            A.gB[fidx] = ea * aj * log(vT);
            vb = ea * aj * qv / vT;
            acc0 -= (double)(ea * aj * pv / uT) * (double)u / (s * s);
          } else {
            vb = kt;
          }
          acc0 += (double)vb * (double)v;
          A.gB[fidx] += ss * vb * v / qv;
          nv[rr] = -ss * vb * v * v / qv;
        }
      }
      X[pr * N + c] = {nv[0], eq ? (T)0 : nv[1]};
    }
  } else if (mode == ROW_ADJU_V1 || mode == ROW_ADJU_B || mode == ROW_ADJU_A) {
    // Reverse sweep of the unbalanced iteration (see adjoint notes above).
    // gk[3 it + {0,1,2}] = (g_k, S_A, S_B) of the iteration being reversed.
    const double G = A.gk[3 * it], SA = A.gk[3 * it + 1], SB = A.gk[3 * it + 2];
    const T Gt = (T)G;
    const T* uh = ubuf_of(A, 0) + I.foff;  // u-hat_k
    const T* vh = vbuf_of(A, 0) + I.foff;  // v-hat_k
    const T ea = (T)I.eps, lam = (T)I.lam, eta = (T)I.eot, tau = (T)I.tau;
    const bool last = (A.k == A.kT);
    T sAb = (T)0, sBb = (T)0;
    if (mode != ROW_ADJU_V1) {
      double gb = 0.0;
      for (int q = tid; q < h; q += bs) gb += A.adjp[(size_t)it * A.hs + q];
      gb = block_sum(gb, sh);
      sAb = (T)(-gb * G / (2.0 * I.eot * SA));
      sBb = (T)(gb * G / (2.0 * I.eot * SB));
    }
    for (int idx = tid; idx < np * N; idx += bs) {
      ROW_PAIR_SETUP(idx)
      const cpx<T> z = has_inverse ? X[pr * N + c] : cpx<T>{(T)0, (T)0};
      T nv[2] = {(T)0, (T)0};
      for (int rr = 0; rr < (eq ? 1 : 2); ++rr) {
        const long long fidx = (rr ? r2 : r1) + c;
        const long long fi = fidx - I.foff;
        const T kt = aj * (rr ? z.y : z.x);  // K^T applied: a (.) (synthesised field)
        if (mode == ROW_ADJU_V1) {
          const T v = vh[fi];
          T vb;
          if (last) {
            const T u = uh[fi], pv = P[fidx], qv = Q[fidx];
            const T uT = u / Gt, vT = Gt * v;
            const T ubT = ea * aj * pv * pow(uT, -eta - (T)1);
            vb = ea * aj * qv * pow(vT, -eta - (T)1);
            acc0 -= (double)ubT * (double)u / (G * G);
            A.gA[fidx] = tau * aj * ((T)1 - pow(uT, -eta));  // direct terms of the cost
            A.gB[fidx] = tau * aj * ((T)1 - pow(vT, -eta));
          } else {
            vb = kt;
          }
          acc0 += (double)vb * (double)v;
          A.vbar[fidx] = vb;
        } else if (mode == ROW_ADJU_B) {
          const T v = vh[fi], qv = Q[fidx];
          const T vhb = Gt * A.vbar[fidx] - eta * sBb * aj * qv * pow(v, -eta - (T)1);
          A.gB[fidx] += sBb * aj * pow(v, -eta) + lam * vhb * v / qv;
          nv[rr] = -lam * vhb * v * pow(v, (T)1 / lam) / qv;
        } else {
          const T u = uh[fi], pv = P[fidx];
          T uhb = kt - eta * sAb * aj * pv * pow(u, -eta - (T)1);
          if (last) uhb += ea * aj * pv * pow(u / Gt, -eta - (T)1) / Gt;
          A.gA[fidx] += sAb * aj * pow(u, -eta) + lam * uhb * u / pv;
          nv[rr] = -lam * uhb * u * pow(u, (T)1 / lam) / pv;
        }
      }
      X[pr * N + c] = {nv[0], eq ? (T)0 : nv[1]};
    }
  } else {  // ROW_FWD, ROW_INIT: load the input rows
    const T* in = A.in;
    for (int idx = tid; idx < np * N; idx += bs) {
      ROW_PAIR_SETUP(idx)
      const T v1 = in ? in[r1 + c] : (T)1;
      const T v2 = eq ? (T)0 : (in ? in[r2 + c] : (T)1);
      X[pr * N + c] = {v1, v2};
      if (mode == ROW_INIT) {
        for (int rr = 0; rr < (eq ? 1 : 2); ++rr) {
          const long long fidx = (rr ? r2 : r1) + c;
          const double pv = P[fidx], qv = Q[fidx];
          acc0 += pv * pv;
          acc1 += (double)aj * pv;
          acc2 += (double)aj * qv;
        }
      }
    }
  }
#undef ROW_PAIR_SETUP

  if (bad) sh_bad = 1;
  if (mode == ROW_INIT) {
    acc0 = block_sum(acc0, sh);
    acc1 = block_sum(acc1, sh);
    acc2 = block_sum(acc2, sh);
    if (tid < np) {
      double* pr = A.prep + ((size_t)it * A.hs + jp0 + tid) * 4;
      pr[0] = tid == 0 ? acc0 : 0.0;
      pr[1] = tid == 0 ? acc1 : 0.0;
      pr[2] = tid == 0 ? acc2 : 0.0;
    }
  } else if (mode == ROW_ADJ_START || mode == ROW_ADJ_VB || mode == ROW_ADJU_V1) {
    acc0 = block_sum(acc0, sh);
    if (tid < np) A.adjp[(size_t)it * A.hs + jp0 + tid] = tid == 0 ? acc0 : 0.0;
    if (mode == ROW_ADJU_V1) return;  // v-bar is consumed pointwise by the next launch
  } else if (mode == ROW_SINK_U || mode == ROW_SINK_V || mode == ROW_CHECK) {
    // residual, kernel range and the half's sum in one block reduction
    __shared__ double sh4[4 * 16];
    double r4[4] = {acc2, kmin, kmax, mode == ROW_SINK_U ? acc0 : acc1};
    block_reduce4(r4, sh4);
    if (A.chk_slot >= 0 && tid < np)
      A.rhist[((size_t)it * A.nslot + A.chk_slot) * A.hs + jp0 + tid] = tid == 0 ? r4[0] : 0.0;
    if (mode != ROW_CHECK) {
      const double kmn = r4[1], kmx = r4[2], s = r4[3];
      // fold the previous half-iteration's kernel ratio into the item's running minimum
      if (A.kr && blockIdx.x == 0) {
        if (mode == ROW_SINK_V) kratio_fold(A, it, A.k, 2, sh);
        else if (A.k > 1) kratio_fold(A, it, A.k - 1, 4, sh);
      }
      if (tid < np) {
        double* rp = A.red + (((size_t)(A.k & 1) * A.nitems_all + it) * A.hs + jp0 + tid) * RED_SLOTS;
        rp[mode == ROW_SINK_U ? 0 : 1] = tid == 0 ? s : 0.0;
        rp[mode == ROW_SINK_U ? 2 : 4] = tid == 0 ? kmn : INFINITY;
        rp[mode == ROW_SINK_U ? 3 : 5] = tid == 0 ? kmx : -INFINITY;
      }
      if (tid == 0 && sh_bad) atomicMin(&A.brk[it], A.k);
    }
    if (mode == ROW_CHECK) return;
  }
  __syncthreads();

  // forward FFT of the rows now in X, fold, weight, store
  cpx<T>* other = (X == buf0) ? buf1 : buf0;
  cpx<T>* Z = RG ? ring_fft<T>(X, other, N, RG, tws, A.ring_blu, (T)-1)
                 : fft_any<T, NC, RPW>(X, other, N, A.fac, A.nfac, tws, (T)-1);
  const bool adj = (mode == ROW_ADJ_START || mode == ROW_ADJ_A || mode == ROW_ADJ_VB || mode == ROW_ADJU_B ||
                   mode == ROW_ADJU_A);
  const bool unweighted = (mode == ROW_FWD && !A.wts_in) || adj;
  for (int idx = tid; idx < np * L; idx += bs) {
    const int m = idx / np, pr = idx - m * np;
    const int jp = jp0 + pr;
    const bool eq = (jp == nlat - 1 - jp);
    const cpx<T>* Zp = Z + pr * N;
    const int cm = RG ? m % N : m;  // HEALPix rings: order m sits in bin m mod N
    const cpx<T> a = Zp[cm];
    cpx<T> b = Zp[(N - cm) % N];
    b.y = -b.y;
    cpx<T> E, O;
    if (eq) {
      E = a;
      O = {(T)0, (T)0};
    } else {
      const cpx<T> x1 = {(T)0.5 * (a.x + b.x), (T)0.5 * (a.y + b.y)};
      const cpx<T> x2 = {(T)0.5 * (a.y - b.y), (T)-0.5 * (a.x - b.x)};
      E = cadd(x1, x2);
      O = csub(x1, x2);
    }
    if (RG) {  // e^{-i m phi0}: the rings' first pixels sit at phi0, not 0
      cpx<T> e = A.ring_ph[(size_t)jp0 * L + m];
      e.y = -e.y;
      E = cmul(E, e);
      O = cmul(O, e);
    }
    const T cw = unweighted ? (T)1 : awl[pr];
    cpx<T>* sp = spec + ((size_t)m * h + jp) * 2;
    sp[0] = cscale(E, cw);
    sp[1] = cscale(O, cw);
  }
}

// ---------------------------------------------------------------------------
// Sinkhorn half-iteration row kernel (modes ROW_SINK_U / ROW_SINK_V), the hot
// path of every solve.  Same arithmetic as row_kernel, organised for latency:
// every global load of the workgroup (spectral gather, marginal, previous u,
// partial sums) is issued before the inverse FFT; the block reductions ride on
// the barriers the FFT needs anyway (wave partials in LDS, combined by one
// thread after the next barrier), so the kernel has two barriers besides the
// FFT stages.  Compile-time transform length NC, BS threads per workgroup.
// ---------------------------------------------------------------------------
template <typename T, int RPW, int NC, int BS>
__global__ void __launch_bounds__(BS) row_sink_kernel(RowArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int N = NC;
  constexpr int NW = BS / 64;
  constexpr int PER = (RPW * N + BS - 1) / BS;  // columns (of both rows of a pair) per thread
  const int L = A.L, h = A.h, nlat = A.nlat;
  cpx<T>* buf0 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* buf1 = buf0 + RPW * N;
  cpx<T>* twl = buf1 + RPW * N;
  __shared__ double shw[NW][4];   // start: gauge sums (0, 1) and previous-half min/max (2, 3)
  __shared__ double shr[NW][4];   // end: sum, residual, min, max of this half
  __shared__ int sh_bad;
  __shared__ T awl[RPW];

  const int ngroups = (h + RPW - 1) / RPW;
  const int jp0 = xcd_row_pair(blockIdx.x, ngroups) * RPW;
  const int np = min(RPW, h - jp0);
  const int it = A.item0 + blockIdx.y;
  const ItemDev I = A.items[it];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mode = A.mode;
  const bool umode = (mode == ROW_SINK_U);
  cpx<T>* spec = A.spec + I.soff;
  const T* F = static_cast<const T*>(umode ? I.p : I.q);  // marginal of this half
  const bool chk = umode && A.chk_slot >= 0;
  const T* uo = ubuf_of(A, A.k - 1) + I.foff;
  T* outf = (umode ? ubuf_of(A, A.k) : vbuf_of(A, A.k)) + I.foff;
  const bool gsum = umode && !A.gk && A.k > 1;       // gauge from the previous iteration's partials
  const bool kfold = A.kr && blockIdx.x == 0 && (!umode || A.k > 1);
  if (tid < RPW) awl[tid] = (tid < np) ? A.aw[jp0 + tid] : (T)0;
  if (tid == 0) sh_bad = 0;

  // Every global load of the group is issued before anything waits on one:
  // unconditional loads at in-bounds addresses into registers (entries the
  // group does not own are loaded from a valid row and never used), then the
  // LDS writes.  A load under a branch makes the join wait for it, which
  // chained the loads into one memory round trip each.
  // (1) field values for the pointwise step (pairs beyond np and the
  // equator's second row are skipped there)
  T fv[PER][2], uv[PER][2];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int idx = tid + e * BS;
    const int pr = min(idx / N, np - 1), c = idx % N;
    const int jp = jp0 + pr, j2 = nlat - 1 - jp;
    const long long r1 = I.foff + (long long)jp * N + c, r2 = I.foff + (long long)j2 * N + c;
    fv[e][0] = __builtin_nontemporal_load(F + r1);
    fv[e][1] = __builtin_nontemporal_load(F + r2);
    uv[e][0] = uv[e][1] = (T)0;
    if (chk) {
      uv[e][0] = __builtin_nontemporal_load(uo + (r1 - I.foff));
      uv[e][1] = __builtin_nontemporal_load(uo + (r2 - I.foff));
    }
  }
  // (2) partial sums of the previous iteration (gauge) and of the previous
  // half (kernel range), one row pair per thread when h <= BS
  double s0 = 0.0, s1 = 0.0, mn = INFINITY, mx = -INFINITY;
  const double* Rg = A.red + ((size_t)((A.k - 1) & 1) * A.nitems_all + it) * (size_t)A.hs * RED_SLOTS;
  const double* Rk = A.red + ((size_t)((umode ? A.k - 1 : A.k) & 1) * A.nitems_all + it) * (size_t)A.hs * RED_SLOTS;
  const int ks = umode ? 4 : 2;
  const bool one_pass = h <= BS;
  const int qp = min(tid, h - 1);
  if (one_pass && gsum) {
    s0 = Rg[(size_t)qp * RED_SLOTS + 0];
    s1 = Rg[(size_t)qp * RED_SLOTS + 1];
  }
  if (one_pass && kfold) {
    mn = Rk[(size_t)qp * RED_SLOTS + ks];
    mx = Rk[(size_t)qp * RED_SLOTS + ks + 1];
  }
  // (3) twiddles and the pairs' spectral entries (L <= (N + 1) / 2 orders)
  constexpr int TI = (N + BS - 1) / BS;
  constexpr int GI = (RPW * ((N + 1) / 2) + BS - 1) / BS;
  cpx<T> twv[TI], ge[GI], go[GI];
#pragma unroll
  for (int i = 0; i < TI; ++i) twv[i] = A.tw[min(tid + i * BS, N - 1)];
  if (!A.cut) {
#pragma unroll
    for (int gi = 0; gi < GI; ++gi) {
      const int idx = tid + gi * BS;
      const int m = idx / RPW, pr = idx - m * RPW;
      const bool ok = m < L && pr < np;
      const cpx<T>* sp = spec + ((size_t)(ok ? m : 0) * h + jp0 + (ok ? pr : 0)) * 2;
      ge[gi] = sp[0];
      go[gi] = sp[1];
    }
  }
  for (int idx = tid; idx < RPW * (N - 2 * L + 1); idx += BS) {
    const int pr = idx / (N - 2 * L + 1), c = L + idx % (N - 2 * L + 1);
    buf0[pr * N + c] = {(T)0, (T)0};
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
    if (tid + i * BS < N) twl[tid + i * BS] = twv[i];
  // Hermitian spectrum of the pair: Z[m] = G_j[m] + i G_j'[m], Z[N-m] its mirror
  auto put = [&](int m, int pr, cpx<T> e, cpx<T> o) {
    const int jp = jp0 + pr;
    const bool eq = (jp == nlat - 1 - jp);
    const cpx<T> a = cadd(e, o);
    const cpx<T> b = eq ? cpx<T>{(T)0, (T)0} : csub(e, o);
    buf0[pr * N + m] = {a.x - b.y, a.y + b.x};
    if (m > 0) buf0[pr * N + N - m] = {a.x + b.y, -a.y + b.x};
  };
  if (!A.cut) {
#pragma unroll
    for (int gi = 0; gi < GI; ++gi) {
      const int idx = tid + gi * BS;
      const int m = idx / RPW, pr = idx - m * RPW;
      if (m < L) put(m, pr, pr < np ? ge[gi] : cpx<T>{(T)0, (T)0}, pr < np ? go[gi] : cpx<T>{(T)0, (T)0});
    }
  } else {
    for (int idx = tid; idx < RPW * L; idx += BS) {
      const int m = idx / RPW, pr = idx - m * RPW;
      cpx<T> e = {(T)0, (T)0}, o = {(T)0, (T)0};
      if (pr < np) load_spec_pair(A, spec, it, m, jp0 + pr, e, o);
      put(m, pr, e, o);
    }
  }
  if (!one_pass)
    for (int q = tid; q < h; q += BS) {
      if (gsum) {
        s0 += Rg[(size_t)q * RED_SLOTS + 0];
        s1 += Rg[(size_t)q * RED_SLOTS + 1];
      }
      if (kfold) {
        mn = fmin(mn, Rk[(size_t)q * RED_SLOTS + ks]);
        mx = fmax(mx, Rk[(size_t)q * RED_SLOTS + ks + 1]);
      }
    }
  else if (tid >= h) {
    s0 = s1 = 0.0;
    mn = INFINITY;
    mx = -INFINITY;
  }
  if (gsum) {
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
  }
  if (kfold) {
    mn = wave_min(mn);
    mx = wave_max(mx);
  }
  if (lane == 0) {
    shw[wave][0] = s0;
    shw[wave][1] = s1;
    shw[wave][2] = mn;
    shw[wave][3] = mx;
  }
  __syncthreads();
  cpx<T>* X = fft_any<T, NC, RPW>(buf0, buf1, N, A.fac, A.nfac, twl, (T)1);

  // (4) gauge (every thread combines the wave sums in wave order)
  double g = 1.0;
  if (umode) {
    if (A.gk) {
      g = A.gk[it];
    } else if (A.k > 1) {
      double s0 = 0.0, s1 = 0.0;
      for (int w = 0; w < NW; ++w) {
        s0 += shw[w][0];
        s1 += shw[w][1];
      }
      g = I.balanced ? s0 : exp(-(0.5 * I.tau * (log(s0) - log(s1))) / I.eps);
    }
  }
  const T gs = (T)g;

  // (5) pointwise update
  double acc = 0.0, acc2 = 0.0, kmin = INFINITY, kmax = -INFINITY;
  bool bad = false;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int idx = tid + e * BS;
    const int pr = idx / N, c = idx - pr * N;
    if (pr >= np) continue;
    const int jp = jp0 + pr;
    const bool eq = (jp == nlat - 1 - jp);
    const T aj = awl[pr];
    const cpx<T> z = X[pr * N + c];
    T nv[2] = {(T)0, (T)0};
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      if (rr && eq) break;
      const T kraw = rr ? z.y : z.x;
      const T f = fv[e][rr];
      if (chk) {
        const double r = (double)uv[e][rr] * (double)kraw - (double)f;
        acc2 += r * r;
      }
      const T kv = umode ? gs * kraw : kraw;
      bad |= bad_kernel_value(kv);
      track_minmax(kmin, kmax, kraw);
      // f / kv from the hardware reciprocal and one Newton step (about 1 ulp;
      // an IEEE divide takes about ten instructions: 13.97 -> 13.83 us per launch)
      const T r0 = __builtin_amdgcn_rcpf(kv);
      const T r1 = fmaf(fmaf(-kv, r0, (T)1), r0, r0);
      T x = f * r1;
      // below the smallest normal float the hardware reciprocal returns inf
      // and the Newton step NaN, where the quotient itself is large but
      // finite: take the IEEE divide there (a branch no lane takes is skipped)
      if (!(kv >= FLT_MIN)) x = f / kv;
      if (!I.balanced) {
        double gt;
        x = unbalanced_update(x, I.lam, I.eot, gt);
        acc += (double)aj * (double)f * gt;
      } else if (umode) {
        acc += (double)x;
      }
      nv[rr] = x;
      const int jr = rr ? nlat - 1 - jp : jp;
      if (A.store_field) __builtin_nontemporal_store(x, outf + (long long)jr * N + c);
    }
    X[pr * N + c] = {nv[0], nv[1]};
  }
  if (umode || !I.balanced) acc = wave_sum(acc);  // balanced V halves keep no sum
  if (chk) acc2 = wave_sum(acc2);
  kmin = wave_min(kmin);
  kmax = wave_max(kmax);
  if (lane == 0) {
    shr[wave][0] = acc;
    shr[wave][1] = acc2;
    shr[wave][2] = kmin;
    shr[wave][3] = kmax;
  }
  if (bad) sh_bad = 1;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0, s2 = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int w = 0; w < NW; ++w) {
      s += shr[w][0];
      s2 += shr[w][1];
      mn = fmin(mn, shr[w][2]);
      mx = fmax(mx, shr[w][3]);
    }
    for (int pr = 0; pr < np; ++pr) {
      double* rp = A.red + (((size_t)(A.k & 1) * A.nitems_all + it) * A.hs + jp0 + pr) * RED_SLOTS;
      rp[umode ? 0 : 1] = pr == 0 ? s : 0.0;
      rp[umode ? 2 : 4] = pr == 0 ? mn : INFINITY;
      rp[umode ? 3 : 5] = pr == 0 ? mx : -INFINITY;
      if (chk) A.rhist[((size_t)it * A.nslot + A.chk_slot) * A.hs + jp0 + pr] = pr == 0 ? s2 : 0.0;
    }
    if (sh_bad) atomicMin(&A.brk[it], A.k);
    if (kfold) {
      double pmn = INFINITY, pmx = -INFINITY;
      for (int w = 0; w < NW; ++w) {
        pmn = fmin(pmn, shw[w][2]);
        pmx = fmax(pmx, shw[w][3]);
      }
      const double r = (pmx > 0.0 && isfinite(pmn)) ? pmn / pmx : -INFINITY;
      A.kr[it] = fmin(A.kr[it], r);
    }
  }

  // (6) forward FFT of the updated rows, fold, weight, store
  cpx<T>* Z = fft_any<T, NC, RPW>(X, X == buf0 ? buf1 : buf0, N, A.fac, A.nfac, twl, (T)-1);
  for (int idx = tid; idx < np * L; idx += BS) {
    const int m = idx / np, pr = idx - m * np;
    const int jp = jp0 + pr;
    const bool eq = (jp == nlat - 1 - jp);
    const cpx<T>* Zp = Z + pr * N;
    const cpx<T> a = Zp[m];
    cpx<T> b = Zp[(N - m) % N];
    b.y = -b.y;
    cpx<T> E, O;
    if (eq) {
      E = a;
      O = {(T)0, (T)0};
    } else {
      const cpx<T> x1 = {(T)0.5 * (a.x + b.x), (T)0.5 * (a.y + b.y)};
      const cpx<T> x2 = {(T)0.5 * (a.y - b.y), (T)-0.5 * (a.x - b.x)};
      E = cadd(x1, x2);
      O = csub(x1, x2);
    }
    const T cw = awl[pr];
    cpx<T>* sp = spec + ((size_t)m * h + jp) * 2;
    sp[0] = cscale(E, cw);
    sp[1] = cscale(O, cw);
  }
}

// ---------------------------------------------------------------------------
// Legendre kernels.  grid = (L orders, item chunks), block = 256.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long tri_off(long long m, long long L) { return m * L - m * (m - 1) / 2; }

template <typename TT>
__device__ __forceinline__ auto tab_load(const TT* p) {
  if constexpr (sizeof(TT) == 2) {
    return __uint_as_float(((unsigned int)(*reinterpret_cast<const unsigned short*>(p))) << 16);
  } else {
    return *p;
  }
}

template <typename T, int IB>
__device__ __forceinline__ void wave_reduce_cpx(cpx<T>* acc) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      acc[i].x += __shfl_xor(acc[i].x, o, 64);
      acc[i].y += __shfl_xor(acc[i].y, o, 64);
    }
  }
}

template <typename T, typename TT, int IB>
__global__ void __launch_bounds__(256) legendre_table_kernel(LegArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = A.L, h = A.h, hpad = A.hpad;
  const int m = blockIdx.x;
  const int ib0 = blockIdx.y * IB;
  const int nbi = min(IB, A.nb - ib0);
  const int nr = L - m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  cpx<T>* ys = reinterpret_cast<cpx<T>*>(smem_raw);  // [IB][2h]
  cpx<T>* bsh = ys + (size_t)IB * 2 * h;              // [IB][L]
  const TT* tab = static_cast<const TT*>(A.tab) + tri_off(m, L) * hpad;
  const long long toff = tri_off(m, L);

  if (A.mode != 2) {
    for (int i = 0; i < IB; ++i) {
      const cpx<T>* src = (i < nbi) ? A.spec + A.items[A.item0 + ib0 + i].soff + (size_t)(2 * m) * h : nullptr;
      for (int idx = tid; idx < 2 * h; idx += blockDim.x)
        ys[(size_t)i * 2 * h + idx] = src ? src[idx] : cpx<T>{(T)0, (T)0};
    }
    __syncthreads();
    for (int r = wave; r < nr; r += nw) {
      const int par = r & 1;
      cpx<T> acc[IB];
#pragma unroll
      for (int i = 0; i < IB; ++i) acc[i] = {(T)0, (T)0};
      const TT* row = tab + (size_t)r * hpad;
      for (int j = lane; j < h; j += 64) {
        const T t = (T)tab_load(row + j);
#pragma unroll
        for (int i = 0; i < IB; ++i) {
          const cpx<T> y = ys[(size_t)i * 2 * h + 2 * j + par];
          acc[i].x += t * y.x;
          acc[i].y += t * y.y;
        }
      }
      wave_reduce_cpx<T, IB>(acc);
      if (lane == 0) {
        for (int i = 0; i < nbi; ++i) {
          if (A.mode == 0) {
            const T hv = A.hl[(size_t)(A.item0 + ib0 + i) * A.hl_stride + m + r];
            bsh[(size_t)i * L + r] = cscale(acc[i], hv);
          } else {
            A.coeff[A.items[A.item0 + ib0 + i].coff + toff + r] = acc[i];
          }
        }
      }
    }
    if (A.mode == 1) return;
  } else {
    for (int i = 0; i < nbi; ++i)
      for (int r = tid; r < nr; r += blockDim.x)
        bsh[(size_t)i * L + r] = A.coeff[A.items[A.item0 + ib0 + i].coff + toff + r];
  }
  __syncthreads();

  for (int j = tid; j < h; j += blockDim.x) {
    cpx<T> ae[IB], ao[IB];
#pragma unroll
    for (int i = 0; i < IB; ++i) { ae[i] = {(T)0, (T)0}; ao[i] = {(T)0, (T)0}; }
    int r = 0;
    for (; r + 1 < nr; r += 2) {
      const T t0 = (T)tab_load(tab + (size_t)r * hpad + j);
      const T t1 = (T)tab_load(tab + (size_t)(r + 1) * hpad + j);
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        const cpx<T> b0 = bsh[(size_t)i * L + r], b1 = bsh[(size_t)i * L + r + 1];
        ae[i].x += t0 * b0.x; ae[i].y += t0 * b0.y;
        ao[i].x += t1 * b1.x; ao[i].y += t1 * b1.y;
      }
    }
    if (r < nr) {
      const T t0 = (T)tab_load(tab + (size_t)r * hpad + j);
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        const cpx<T> b0 = bsh[(size_t)i * L + r];
        ae[i].x += t0 * b0.x; ae[i].y += t0 * b0.y;
      }
    }
    for (int i = 0; i < nbi; ++i) {
      cpx<T>* dst = A.spec + A.items[A.item0 + ib0 + i].soff + (size_t)(2 * m) * h;
      dst[2 * j] = ae[i];
      dst[2 * j + 1] = ao[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Legendre kernel with P̄_l^m generated on the fly (float64 recurrence).
//
// Each thread owns JPT latitude chains j.  The recurrence is the rescaled
// three-term form R_l = c_l x R_{l-1} + R_{l-2}, P̄_l^m = gamma_l R_l (two
// float64 operations per value; c_l and gamma_l are precomputed on the host),
// restarted from the seed P̄_m^m(x_j) for the synthesis pass.  Products and
// per-lane accumulations are float64.  Analysis sums over j are formed per
// block of RB rows: a wave transpose-reduction (permlane swaps for the two
// upper lane bits, DPP mirrors/quad permutes below) leaves value v = lane/2
// summed over the wave; waves are combined through LDS in wave order, one
// barrier per block (double-buffered partials).  Coefficients and spectral
// inputs are staged in LDS, zero-padded to whole blocks so the row loops need
// no bounds tests.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R dpp_any(R v, int sel) {
  if constexpr (sizeof(R) == 4) return dpp_f(v, sel);
  else return dpp_d(v, sel);
}

// NV (16 or 32) values per lane -> lane L holds the wave sum of value
// L >> (6 - log2 NV): each stage halves the values a lane keeps while doubling
// the lanes summed, so NV - 1 adds and exchanges in total.
template <typename R, int NV>
__device__ __forceinline__ R transpose_reduce(R* a, int lane) {
  static_assert(NV == 16 || NV == 32, "NV");
#pragma unroll
  for (int i = 0; i < NV / 2; ++i) a[i] = swap_add32(a[i], a[NV / 2 + i]);   // lane bit 5
#pragma unroll
  for (int i = 0; i < NV / 4; ++i) a[i] = swap_add16(a[i], a[NV / 4 + i]);   // lane bit 4
  {
    const bool up = (lane & 8) != 0;                                          // lane bit 3
#pragma unroll
    for (int i = 0; i < NV / 8; ++i) {
      const R send = up ? a[i] : a[NV / 8 + i];
      const R keep = up ? a[NV / 8 + i] : a[i];
      a[i] = keep + dpp_any(send, 0);
    }
  }
  {
    const bool up = (lane & 4) != 0;                                          // lane bit 2
#pragma unroll
    for (int i = 0; i < NV / 16; ++i) {
      const R send = up ? a[i] : a[NV / 16 + i];
      const R keep = up ? a[NV / 16 + i] : a[i];
      a[i] = keep + dpp_any(send, 1);
    }
  }
  if constexpr (NV == 32) {
    const bool up = (lane & 2) != 0;                                          // lane bit 1
    const R send = up ? a[0] : a[1];
    const R keep = up ? a[1] : a[0];
    a[0] = keep + dpp_any(send, 2);
  } else {
    a[0] += dpp_any(a[0], 2);
  }
  a[0] += dpp_any(a[0], 3);                                                   // lane bit 0
  return a[0];
}

// 32 values per lane -> lane L holds the wave sum of value (L >> 1).
template <typename R>
__device__ __forceinline__ R transpose_reduce32(R* a, int lane) {
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = swap_add32(a[i], a[16 + i]);   // lane bit 5
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = swap_add16(a[i], a[8 + i]);     // lane bit 4
  {
    const bool up = (lane & 8) != 0;                                  // lane bit 3
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const R send = up ? a[i] : a[4 + i];
      const R keep = up ? a[4 + i] : a[i];
      a[i] = keep + dpp_any(send, 0);
    }
  }
  {
    const bool up = (lane & 4) != 0;                                  // lane bit 2
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const R send = up ? a[i] : a[2 + i];
      const R keep = up ? a[2 + i] : a[i];
      a[i] = keep + dpp_any(send, 1);
    }
  }
  {
    const bool up = (lane & 2) != 0;                                  // lane bit 1
    const R send = up ? a[0] : a[1];
    const R keep = up ? a[1] : a[0];
    a[0] = keep + dpp_any(send, 2);
  }
  a[0] += dpp_any(a[0], 3);                                           // lane bit 0
  return a[0];
}

template <typename T, int IB, int JPT>
__global__ void __launch_bounds__(256) legendre_recur_kernel(LegArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using R = T;                       // reduction type: float for float32 plans
  constexpr int RB = 16 / IB;        // rows per block
  constexpr int V = 2 * RB * IB;     // 32 partial sums per lane per block
  const int L = A.L, h = A.h;
  const int m = blockIdx.x;
  const int nr = L - m;
  const int nblk = (nr + RB - 1) / RB;
  const int npad = nblk * RB;
  const int ib0 = blockIdx.y * IB;
  const int nbi = min(IB, A.nb - ib0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6, nt = blockDim.x;
  // LDS: cf[npad], gm[npad] (double), b[IB][npad] (double2), part[2][nw][V] (R)
  double* cf = reinterpret_cast<double*>(smem_raw);
  double* gm = cf + npad;
  double2* bs = reinterpret_cast<double2*>(gm + npad);
  R* part = reinterpret_cast<R*>(bs + (size_t)IB * npad);
  const long long toff = tri_off(m, L);

  for (int r = tid; r < npad; r += nt) {
    cf[r] = (r < nr && r > 0) ? A.rcoef[toff + r] : 0.0;
    gm[r] = (r < nr) ? A.rgam[toff + r] : 0.0;
  }
  for (int i = 0; i < IB; ++i)
    for (int r = tid; r < npad; r += nt) bs[(size_t)i * npad + r] = make_double2(0.0, 0.0);

  double xj[JPT], R1[JPT], R2[JPT], seed[JPT];
  double2 yE[JPT][IB], yO[JPT][IB];
#pragma unroll
  for (int c = 0; c < JPT; ++c) {
    const int j = tid + c * nt;
    const bool act = j < h;
    xj[c] = act ? A.xs[j] : 0.0;
    seed[c] = act ? A.rseed[(size_t)m * h + j] : 0.0;
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      yE[c][i] = make_double2(0.0, 0.0);
      yO[c][i] = make_double2(0.0, 0.0);
      if (act && i < nbi && A.mode != 2) {
        const cpx<T>* s = A.spec + A.items[A.item0 + ib0 + i].soff + (size_t)(2 * m) * h;
        const cpx<T> e = s[2 * j], o = s[2 * j + 1];
        yE[c][i] = make_double2((double)e.x, (double)e.y);
        yO[c][i] = make_double2((double)o.x, (double)o.y);
      }
    }
  }
  __syncthreads();

  if (A.mode != 2) {
#pragma unroll
    for (int c = 0; c < JPT; ++c) { R1[c] = seed[c]; R2[c] = 0.0; }
    for (int blk = 0; blk < nblk; ++blk) {
      const int r0 = blk * RB;
      double acc[V];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = 0.0;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const double c0 = cf[r0 + rr];
#pragma unroll
        for (int c = 0; c < JPT; ++c) {
          if (r0 + rr > 0) {
            const double rn = fma(c0 * xj[c], R1[c], R2[c]);
            R2[c] = R1[c];
            R1[c] = rn;
          }
#pragma unroll
          for (int i = 0; i < IB; ++i) {
            const double2 y = (rr & 1) ? yO[c][i] : yE[c][i];  // r0 is even
            acc[(rr * IB + i) * 2 + 0] = fma(R1[c], y.x, acc[(rr * IB + i) * 2 + 0]);
            acc[(rr * IB + i) * 2 + 1] = fma(R1[c], y.y, acc[(rr * IB + i) * 2 + 1]);
          }
        }
      }
      R red[V];
#pragma unroll
      for (int v = 0; v < V; ++v) red[v] = (R)acc[v];
      const R s = transpose_reduce32<R>(red, lane);
      R* pb = part + (size_t)(blk & 1) * nw * V;
      if ((lane & 1) == 0) pb[wave * V + (lane >> 1)] = s;
      __syncthreads();
      if (tid < V) {
        double tot = 0.0;
        for (int w = 0; w < nw; ++w) tot += (double)pb[w * V + tid];
        const int comp = tid & 1, i = (tid >> 1) % IB, rr = (tid >> 1) / IB, r = r0 + rr;
        if (r < nr && i < nbi) {
          const double g = gm[r];
          if (A.mode == 0) {
            const double sc = g * g * (double)A.hl[(size_t)(A.item0 + ib0 + i) * A.hl_stride + m + r];
            double* dst = reinterpret_cast<double*>(&bs[(size_t)i * npad + r]);
            dst[comp] = tot * sc;
          } else {
            T* dst = reinterpret_cast<T*>(&A.coeff[A.items[A.item0 + ib0 + i].coff + toff + r]);
            dst[comp] = (T)(tot * g);
          }
        }
      }
    }
    if (A.mode == 1) return;
  } else {
    for (int i = 0; i < nbi; ++i)
      for (int r = tid; r < nr; r += nt) {
        const cpx<T> c = A.coeff[A.items[A.item0 + ib0 + i].coff + toff + r];
        bs[(size_t)i * npad + r] = make_double2((double)c.x * gm[r], (double)c.y * gm[r]);
      }
  }
  __syncthreads();

  // synthesis: G^{E|O}_m(j) = sum_l (b_l gamma_l) R_l(x_j), rows in blocks of 16
  double2 gE[JPT][IB], gO[JPT][IB];
#pragma unroll
  for (int c = 0; c < JPT; ++c) {
    R1[c] = seed[c];
    R2[c] = 0.0;
#pragma unroll
    for (int i = 0; i < IB; ++i) { gE[c][i] = make_double2(0.0, 0.0); gO[c][i] = make_double2(0.0, 0.0); }
  }
  const int nblk16 = (nr + 15) / 16;
  for (int blk = 0; blk < nblk16; ++blk) {
    const int r0 = blk * 16;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int r = r0 + rr;
      const double c0 = (r < npad) ? cf[r] : 0.0;
      double2 b[IB];
#pragma unroll
      for (int i = 0; i < IB; ++i) b[i] = (r < npad) ? bs[(size_t)i * npad + r] : make_double2(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < JPT; ++c) {
        if (r > 0) {
          const double rn = fma(c0 * xj[c], R1[c], R2[c]);
          R2[c] = R1[c];
          R1[c] = rn;
        }
#pragma unroll
        for (int i = 0; i < IB; ++i) {
          if (rr & 1) {
            gO[c][i].x = fma(R1[c], b[i].x, gO[c][i].x);
            gO[c][i].y = fma(R1[c], b[i].y, gO[c][i].y);
          } else {
            gE[c][i].x = fma(R1[c], b[i].x, gE[c][i].x);
            gE[c][i].y = fma(R1[c], b[i].y, gE[c][i].y);
          }
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < JPT; ++c) {
    const int j = tid + c * nt;
    if (j >= h) continue;
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      if (i >= nbi) continue;
      cpx<T>* dst = A.spec + A.items[A.item0 + ib0 + i].soff + (size_t)(2 * m) * h;
      dst[2 * j] = {(T)gE[c][i].x, (T)gE[c][i].y};
      dst[2 * j + 1] = {(T)gO[c][i].x, (T)gO[c][i].y};
    }
  }
}

// ---------------------------------------------------------------------------
// Row-split recurrence Legendre kernel.
//
// One workgroup (4 waves) per part of an order m (rows [r_lo, r_hi) of the
// order, taken from a host work list in a host-chosen dispatch order) and
// item chunk.  Every
// lane owns the C latitude chains j = lane + 64 c, and the part's rows are
// split into four contiguous ranges, one per wave.  A wave resumes the
// rescaled recurrence at the start of its range from a plan-time checkpoint
// (R_{r0}, R_{r0-1}).  Analysis sums over j are complete within a wave (C
// chains per lane, then a wave transpose-reduction), so the analysis loop has
// no barrier and a part needs no other part's analysis.  Synthesis partial
// sums of the four waves are combined once through LDS; an order cut into
// several parts (so that long orders spread over several compute units) has
// each part store its sum to a partial buffer; the consumer adds the parts in
// part order, which keeps the result independent of timing.
// ---------------------------------------------------------------------------

// A copy of a lane-varying index that the compiler cannot see through: the
// addresses derived from it are recomputed where they are used instead of
// being shared with (and kept live across the loops until) a later use of the
// same expression.
__device__ __forceinline__ int opaque_index(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Wave issue priority from the blocks of rows a wave still has to run (both
// passes): the three waves sharing a SIMD come from different orders, and
// running the one with the most work left first makes them finish together
// instead of leaving one long wave alone on the SIMD at the end.  Thresholds
// from interleaved timings at L = 720 (priorities off 41.4 us, on 39.5; with
// the current dispatch packing 12/6/2 beats 14/7/2, 10/5/2 and 16/8/3).
__device__ __forceinline__ void prio_by_blocks(int left) {
  if (left >= 12) __builtin_amdgcn_s_setprio(3);
  else if (left >= 6) __builtin_amdgcn_s_setprio(2);
  else if (left >= 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// Three waves per SIMD where the registers allow it without spilling: then
// a launch of up to 3 x 256 workgroups is resident at once, and the host's
// dispatch order balances the rows that meet on one compute unit.
template <typename T, int IB, int C, int NV>
__global__ void __launch_bounds__(256, IB * C > 6 ? 2 : 3) legendre_split_kernel(LegArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using R = T;
  constexpr int RB = NV / (2 * IB);
  constexpr int V = NV;
  const int L = A.L, h = A.h;
  const int part = blockIdx.x;  // the work list is stored in dispatch order
  const SplitPartH P = A.parts[part];
  const int m = P.m;
  const int nr = L - m;
  const int len = P.r_hi - P.r_lo;
  const int npl = (len + 15) / 16 * 16 + 16;  // one extra block: the look-ahead coefficient
  const int ib0 = blockIdx.y * IB;
  const int nbi = min(IB, A.nb - ib0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: row range in scalars
  const int maxpl = (A.maxlen + 15) / 16 * 16 + 16;
  double* cf = reinterpret_cast<double*>(smem_raw);                   // [maxpl], local row index
  double* gm = cf + maxpl;
  double2* bs = reinterpret_cast<double2*>(gm + maxpl);               // [IB][maxpl]
  cpx<T>* gpart = reinterpret_cast<cpx<T>*>(bs + (size_t)IB * maxpl);  // [4][IB][h][2]
  const long long toff = tri_off(m, L);
  const int r_lo = P.r_lo + split_row(len, wave), r_hi = P.r_lo + split_row(len, wave + 1);

  // Every global load of the prologue is issued before the first wait:
  // unconditional loads at clamped, in-bounds addresses into registers (values
  // a thread does not own are dropped at the LDS store or replaced at their
  // use).  A load under a branch makes the join wait for it, which chained the
  // coefficient, spectrum and checkpoint loads into one round trip each.
  constexpr int NQ = 3;  // per-thread coefficient rows and spectrum entries staged at once
  const int ptid = opaque_index(tid), plane = ptid & 63;
  long long soff[IB];
#pragma unroll
  for (int i = 0; i < IB; ++i) soff[i] = A.items[A.item0 + ib0 + min(i, nbi - 1)].soff;
  double cv[NQ], gv[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int r = min(P.r_lo + ptid + k * 256, nr - 1);
    cv[k] = A.rcoef[toff + r];
    gv[k] = A.rgam[toff + r];
  }
  cpx<T> sv[IB][NQ];
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int k = 0; k < NQ; ++k)
      sv[i][k] = A.spec[soff[i] + (size_t)(2 * m) * h + min(ptid + k * 256, 2 * h - 1)];
  double xj[C];
#pragma unroll
  for (int c = 0; c < C; ++c) xj[c] = A.xs[min(plane + 64 * c, h - 1)];
  const double2* ckp = reinterpret_cast<const double2*>(A.rck) + ((size_t)part * 4 + wave) * h;
  // the first wave of a part that starts an order resumes from the seed
  // (P̄_m^m, 0) itself: half the bytes of its checkpoint (the second value is
  // then a re-read of the first and replaced by zero)
  const bool from_seed = wave == 0 && P.r_lo == 0;
  auto ck_load = [&](int c, int ln) {
    const int j = min(ln + 64 * c, h - 1);
    const double* p = from_seed ? A.rseed + (size_t)m * h + j : reinterpret_cast<const double*>(ckp + j);
    return make_double2(p[0], p[from_seed ? 0 : 1]);
  };
  auto ck_use = [&](double2 v, int c) {
    const bool ok = lane + 64 * c < h;
    return make_double2(ok ? v.x : 0.0, ok && !from_seed ? v.y : 0.0);
  };
  double2 ck[C];
#pragma unroll
  for (int c = 0; c < C; ++c) ck[c] = ck_load(c, plane);

#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = ptid + k * 256, r = P.r_lo + q;
    if (q < npl) {
      cf[q] = (r < nr && r > 0) ? cv[k] : 0.0;
      gm[q] = (r < nr) ? gv[k] : 0.0;
    }
  }
  for (int q = tid + NQ * 256; q < npl; q += 256) {  // longer parts than one staging round
    const int r = P.r_lo + q;
    cf[q] = (r < nr && r > 0) ? A.rcoef[toff + r] : 0.0;
    gm[q] = (r < nr) ? A.rgam[toff + r] : 0.0;
  }
  for (int i = 0; i < IB; ++i)
    for (int q = tid; q < npl; q += 256) bs[(size_t)i * maxpl + q] = make_double2(0.0, 0.0);
  // this order's folded spectrum, staged once per workgroup in the LDS that
  // the synthesis partial sums reuse later (read into registers before then)
  if (A.mode != 2)
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      if (i >= nbi) break;
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const int q = ptid + k * 256;
        if (q < 2 * h) gpart[(size_t)i * 2 * h + q] = sv[i][k];
      }
      const cpx<T>* src = A.spec + soff[i] + (size_t)(2 * m) * h;
      for (int q = tid + NQ * 256; q < 2 * h; q += 256) gpart[(size_t)i * 2 * h + q] = src[q];
    }
#pragma unroll
  for (int c = 0; c < C; ++c) xj[c] = lane + 64 * c < h ? xj[c] : 0.0;
  __syncthreads();

  if (A.mode != 2) {
    double2 yE[C][IB], yO[C][IB];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = lane + 64 * c;
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        yE[c][i] = make_double2(0.0, 0.0);
        yO[c][i] = make_double2(0.0, 0.0);
        if (j < h && i < nbi) {
          const cpx<T>* s = gpart + (size_t)i * 2 * h;
          const cpx<T> e = s[2 * j], o = s[2 * j + 1];
          yE[c][i] = make_double2((double)e.x, (double)e.y);
          yO[c][i] = make_double2((double)o.x, (double)o.y);
        }
      }
    }
    double R1[C], R2[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double2 v = ck_use(ck[c], c);
      R1[c] = v.x;
      R2[c] = v.y;
    }
    const int nblk = (r_hi - r_lo + RB - 1) / RB;  // this wave's blocks in each of the two passes
    int left = 2 * nblk;
    constexpr int SH = NV == 32 ? 1 : 2;  // lanes per reduced value after the transpose-reduction
    // this lane's heat multiplier for row r0 + (its row in the block): loaded
    // at the start of each block, used after the block's arithmetic (rows past
    // the order's end read the array's padding and are dropped)
    const int hoff = (A.item0 + ib0 + min(((lane >> SH) >> 1) % IB, nbi - 1)) * A.hl_stride + m +
                     ((lane >> SH) >> 1) / IB;
    for (int r0 = r_lo; r0 < r_hi; r0 += RB) {
      prio_by_blocks(left--);
      const T hlv = A.hl[hoff + r0];
      double acc[V];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = 0.0;
      const double* cfr = cf + (r0 - P.r_lo) + 1;  // coefficient of the next row
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const double cn = cfr[rr];
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int i = 0; i < IB; ++i) {
            const double2 y = (rr & 1) ? yO[c][i] : yE[c][i];  // every range starts on an even row
            acc[(rr * IB + i) * 2 + 0] = fma(R1[c], y.x, acc[(rr * IB + i) * 2 + 0]);
            acc[(rr * IB + i) * 2 + 1] = fma(R1[c], y.y, acc[(rr * IB + i) * 2 + 1]);
          }
          const double rn = fma(cn * xj[c], R1[c], R2[c]);
          R2[c] = R1[c];
          R1[c] = rn;
        }
      }
      R red[V];
#pragma unroll
      for (int v = 0; v < V; ++v) red[v] = (R)acc[v];
      const R s = transpose_reduce<R, NV>(red, lane);
      if ((lane & ((1 << SH) - 1)) == 0) {
        const int vv = lane >> SH, comp = vv & 1, i = (vv >> 1) % IB, rr = (vv >> 1) / IB, r = r0 + rr;
        if (r < r_hi && i < nbi) {
          const int q = r - P.r_lo;
          const double g = gm[q];
          if (A.mode == 0) {
            const double sc = g * g * (double)hlv;
            reinterpret_cast<double*>(&bs[(size_t)i * maxpl + q])[comp] = (double)s * sc;
          } else {
            T* dst = reinterpret_cast<T*>(&A.coeff[A.items[A.item0 + ib0 + i].coff + toff + r]);
            dst[comp] = (T)((double)s * g);
          }
        }
      }
    }
    if (A.mode == 1) return;
  } else {
    for (int i = 0; i < nbi; ++i)
      for (int q = tid; q < len; q += 256) {
        const cpx<T> c = A.coeff[A.items[A.item0 + ib0 + i].coff + toff + P.r_lo + q];
        bs[(size_t)i * maxpl + q] = make_double2((double)c.x * gm[q], (double)c.y * gm[q]);
      }
  }
  // the synthesis pass restarts from the same checkpoints: issue their loads
  // before the barrier so that they arrive while the workgroup's waves meet
  {
    const int ln = opaque_index(lane);
#pragma unroll
    for (int c = 0; c < C; ++c) ck[c] = ck_load(c, ln);
  }
  __syncthreads();

  // synthesis over this wave's rows: G^{E|O}_m(j) += (b_l gamma_l) R_l(x_j)
  double2 gE[C][IB], gO[C][IB];
  double R1[C], R2[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const double2 v = ck_use(ck[c], c);
    R1[c] = v.x;
    R2[c] = v.y;
#pragma unroll
    for (int i = 0; i < IB; ++i) { gE[c][i] = make_double2(0.0, 0.0); gO[c][i] = make_double2(0.0, 0.0); }
  }
  int left = (r_hi - r_lo + 15) / 16;
  for (int r0 = r_lo; r0 < r_hi; r0 += 16) {
    prio_by_blocks(left--);
    const int q0 = r0 - P.r_lo;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const double cn = cf[q0 + rr + 1];
      double2 b[IB];
#pragma unroll
      for (int i = 0; i < IB; ++i) b[i] = bs[(size_t)i * maxpl + q0 + rr];
#pragma unroll
      for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int i = 0; i < IB; ++i) {
          if (rr & 1) {
            gO[c][i].x = fma(R1[c], b[i].x, gO[c][i].x);
            gO[c][i].y = fma(R1[c], b[i].y, gO[c][i].y);
          } else {
            gE[c][i].x = fma(R1[c], b[i].x, gE[c][i].x);
            gE[c][i].y = fma(R1[c], b[i].y, gE[c][i].y);
          }
        }
        const double rn = fma(cn * xj[c], R1[c], R2[c]);
        R2[c] = R1[c];
        R1[c] = rn;
      }
    }
  }
  __builtin_amdgcn_s_setprio(0);
  // combine the four waves' partial sums (fixed order)
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int j = lane + 64 * c;
    if (j >= h) continue;
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      cpx<T>* gp = gpart + (((size_t)wave * IB + i) * 2) * h;
      gp[2 * j] = {(T)gE[c][i].x, (T)gE[c][i].y};  // same [j][E/O] order as the spectrum
      gp[2 * j + 1] = {(T)gO[c][i].x, (T)gO[c][i].y};
    }
  }
  __syncthreads();
  if (P.ns == 1) {
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      if (i >= nbi) break;
      cpx<T>* dst = A.spec + soff[i] + (size_t)(2 * m) * h;
      for (int q = tid; q < 2 * h; q += 256) {
        cpx<T> s = {(T)0, (T)0};
#pragma unroll
        for (int w = 0; w < 4; ++w) s = cadd(s, gpart[(((size_t)w * IB + i) * 2) * h + q]);
        dst[q] = s;
      }
    }
    return;
  }
  // order cut into parts: store this part's sum; the row kernel that reads
  // the spectrum next adds the parts of the order in part order
  cpx<T>* pb = static_cast<cpx<T>*>(A.pbuf) + (size_t)blockIdx.y * A.npb * IB * 2 * h;
  for (int i = 0; i < nbi; ++i) {
    cpx<T>* dst = pb + ((size_t)P.pslot * IB + i) * 2 * h;
    for (int q = tid; q < 2 * h; q += 256) {
      cpx<T> s = {(T)0, (T)0};
#pragma unroll
      for (int w = 0; w < 4; ++w) s = cadd(s, gpart[(((size_t)w * IB + i) * 2) * h + q]);
      dst[q] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Batched Legendre stage as matrix-core GEMMs (table plans, many items).
//
// Per order m and parity, with columns n = (item, re/im) of the workgroup:
//   analysis   D[r][n] = sum_j P̄[r][j] Y[j][n]       (A = table rows, K = j)
//   scale      b[r][n] = D[r][n] h_l(item)
//   synthesis  G[j][n] = sum_r P̄T[j][r] b[r][n]      (A = transposed table, K = r)
// on v_mfma_f32_16x16x32_bf16 (bf16 operands) or v_mfma_f32_16x16x4_f32 (fp32
// operands), fp32 accumulation.  Operand layout of the 16x16 MFMAs: A[i][k] in
// lane i + 16*(k/kv), element k%kv; B[k][j] in lane j + 16*(k/kv); D[i][j] in
// lane j + 16*(i/4), register i%4 (kv = 8 for bf16, 1 for fp32).  Y and b are
// staged in LDS as [n][k] rows padded so the 16 lanes of a k-slice hit
// distinct banks.
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}


template <typename TT>
struct MmaTraits;
template <>
struct MmaTraits<unsigned short> {  // bf16
  static constexpr int KS = 32, KV = 8, PAD = 8;
  __device__ static unsigned short cvt(float v) { return f32_to_bf16_rne(v); }
  __device__ static f32x4_t mma(const unsigned short* a, const unsigned short* b, f32x4_t c) {
    const uint4 av = *reinterpret_cast<const uint4*>(a);
    const uint4 bv = *reinterpret_cast<const uint4*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                   __builtin_bit_cast(bf16x8_t, bv), c, 0, 0, 0);
  }
  __device__ static void load_a(unsigned short* dst, const unsigned short* src, bool ok) {
    *reinterpret_cast<uint4*>(dst) = ok ? *reinterpret_cast<const uint4*>(src) : make_uint4(0, 0, 0, 0);
  }
};
template <>
struct MmaTraits<float> {
  static constexpr int KS = 4, KV = 1, PAD = 1;
  __device__ static float cvt(float v) { return v; }
  __device__ static f32x4_t mma(const float* a, const float* b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
  }
  __device__ static void load_a(float* dst, const float* src, bool ok) { *dst = ok ? *src : 0.0f; }
};

// Per-wave synthesis tile of legendre_mma_kernel: 32 table rows x 16 qt
// latitudes, row pitch in elements.  bfloat16 rows of an odd word count = 1
// mod 4 put the four lane groups' rows (8 apart) on distinct banks; float rows
// keep 16-byte alignment.  Eight-wave workgroups take 32-latitude tasks.
// waves per workgroup: eight for a single item (a launch of one workgroup per
// order is otherwise too few waves to keep the table stream in flight)
__host__ __device__ constexpr int mma_waves(bool narrow) { return narrow ? 8 : 4; }
__host__ __device__ constexpr int mma_tile_q(int nw) { return nw == 8 ? 2 : 4; }
__host__ __device__ constexpr int mma_tile_ld(int es, int qt) { return es == 2 ? 16 * qt + 2 : 16 * qt + 4; }
// byte offset of the four tiles: after Y and b, rounded up to 16 bytes
__host__ __device__ inline size_t mma_tile_off(int L, int hpad, int ns, int es, int pad) {
  const size_t yb = (size_t)es * 2 * ns * ((size_t)hpad + pad) + (size_t)es * 2 * ns * (mma_rpad((L + 1) / 2) + pad);
  return (yb + 15) / 16 * 16;
}

template <typename T, typename TT, int NT, bool NARROW, int NW>
__global__ void __launch_bounds__(64 * NW) legendre_mma_kernel(LegArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using MT = MmaTraits<TT>;
  constexpr int NB = 16 * NT, KS = MT::KS, KV = MT::KV;
  // B-operand rows kept in LDS per parity: the tile's NB columns, or, for a
  // single item (NARROW), its two columns and one zero row that the other 14
  // lanes of a k-slice all read (a broadcast): 3 rows instead of 16
  constexpr int NS = NARROW ? 3 : NB;
  auto srow = [](int n) { return NARROW ? (n < 2 ? n : 2) : n; };
  constexpr int KG = sizeof(TT) == 2 ? 8 : 16;  // k-steps whose A operands are loaded together
  const int L = A.L, h = A.h, kpad = A.hpad;
  const int m = A.morder ? A.morder[blockIdx.x] : (int)blockIdx.x, nr = L - m;
  const int c0 = blockIdx.y * NB;
  const int ncol = 2 * A.nb;
  const int RP = mma_rpad((L + 1) / 2);
  const int ys_ld = kpad + MT::PAD, bs_ld = RP + MT::PAD;
  TT* ys = reinterpret_cast<TT*>(smem_raw);                // [2][NS][ys_ld]
  TT* bs = ys + (size_t)2 * NS * ys_ld;                    // [2][NS][bs_ld]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const long long toff = tri_off(m, L);
  const TT* tab = static_cast<const TT*>(A.tab) + toff * kpad;

  // stage Y (zero beyond h and beyond the last column) and clear b: one
  // (parity, column) row per wave at a time, latitudes across the lanes
  for (int pn = wave; pn < 2 * NS; pn += NW) {
    const int par = pn / NS, n = pn - par * NS;
    const int col = c0 + n;  // (the zero row of a NARROW tile: col = 2 >= ncol)
    const bool cok = A.mode != 2 && col < ncol;
    const cpx<T>* sp = A.spec + (cok ? A.items[A.item0 + (col >> 1)].soff : 0) + (size_t)m * h * 2 + par;
    TT* dst = ys + ((size_t)par * NS + n) * ys_ld;
    for (int j = lane; j < kpad; j += 64) {
      float v = 0.f;
      if (cok && j < h) {
        const cpx<T> y = sp[2 * j];
        v = (float)((col & 1) ? y.y : y.x);
      }
      dst[j] = MT::cvt(v);
    }
  }
  for (int idx = tid; idx < 2 * NS * bs_ld; idx += 64 * NW) bs[idx] = MT::cvt(0.f);
  __syncthreads();

  if (A.mode != 2) {
    for (int par = 0; par < 2; ++par) {
      const int npar = (nr + 1 - par) / 2;
      const int Rt = (npar + 15) / 16;
      for (int t = wave; t < Rt; t += NW) {
        f32x4_t acc[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        const int rp = t * 16 + li;          // row (of this parity) fed by this lane
        const int r = 2 * rp + par;
        const bool rok = rp < npar;
        const TT* arow = tab + (size_t)(rok ? r : 0) * kpad + lg * KV;
        // A operands of KG k-steps are fetched together: one memory latency
        // per group instead of one per step
        for (int kg = 0; kg < kpad; kg += KG * KS) {
          TT a[KG][KV];
#pragma unroll
          for (int s = 0; s < KG; ++s) MT::load_a(a[s], arow + kg + s * KS, rok && kg + s * KS < kpad);
#pragma unroll
          for (int s = 0; s < KG; ++s) {
            if (kg + s * KS >= kpad) break;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
              const TT* bp = ys + ((size_t)par * NS + srow(c * 16 + li)) * ys_ld + kg + s * KS + lg * KV;
              acc[c] = MT::mma(a[s], bp, acc[c]);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < NT; ++c) {
          const int n = c * 16 + li, col = c0 + n;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int rpo = t * 16 + lg * 4 + i, ro = 2 * rpo + par;
            if (rpo < npar && col < ncol) {
              const int item = A.item0 + (col >> 1);
              if (A.mode == 0) {
                const float hv = (float)A.hl[(size_t)item * A.hl_stride + m + ro];
                bs[((size_t)par * NS + n) * bs_ld + rpo] = MT::cvt(acc[c][i] * hv);  // n < ncol <= NS
              } else {
                T* dst = reinterpret_cast<T*>(&A.coeff[A.items[item].coff + toff + ro]);
                dst[col & 1] = (T)acc[c][i];
              }
            }
          }
        }
      }
    }
    if (A.mode == 1) return;
  } else {
    for (int idx = tid; idx < NB * nr; idx += 64 * NW) {
      const int n = idx / nr, r = idx % nr, col = c0 + n;
      if (col >= ncol) continue;
      const cpx<T> c = A.coeff[A.items[A.item0 + (col >> 1)].coff + toff + r];
      bs[((size_t)(r & 1) * NS + n) * bs_ld + (r >> 1)] = MT::cvt((float)((col & 1) ? c.y : c.x));
    }
  }
  __syncthreads();

  // Synthesis G[j][n] = sum_r P[r][j] b[r][n] per parity, from the same
  // row-major table as the analysis (no second copy: one stream of the table
  // per launch).  The A operand needs the rows along K, so each wave stages
  // 32 rows x 64 latitudes of one parity in its own LDS tile (coalesced
  // 16-byte loads) and reads the operands across the rows.  Tasks: (parity,
  // 16 QT latitudes), QT 16-latitude tiles per task.
  constexpr int QT = mma_tile_q(NW);
  constexpr int TW = mma_tile_ld(sizeof(TT), QT);
  constexpr int EPL = 16 / sizeof(TT);  // elements per 16-byte load
  constexpr int LPR = 16 * QT / EPL;    // lanes per tile row
  constexpr int RPL = 64 / LPR;         // tile rows per load round
  TT* tw = reinterpret_cast<TT*>(smem_raw + mma_tile_off(L, kpad, NS, sizeof(TT), MT::PAD)) + (size_t)wave * 32 * TW;
  const int Jq = (h + 16 * QT - 1) / (16 * QT);
  for (int task = wave; task < 2 * Jq; task += NW) {
    const int par = task / Jq, jq = task - par * Jq;
    const int npar = (nr + 1 - par) / 2;
    f32x4_t acc[QT][NT];
#pragma unroll
    for (int q = 0; q < QT; ++q)
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[q][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int jl = 16 * QT * jq + (lane % LPR) * EPL;  // first latitude of this lane's loads
    // the next chunk's rows are loaded while this one is contracted
    uint4 v[32 / RPL];
    auto load_chunk = [&](int k0) {
#pragma unroll
      for (int u = 0; u < 32 / RPL; ++u) {
        const int rp = k0 + u * RPL + lane / LPR;
        v[u] = rp < npar && jl < kpad
                   ? *reinterpret_cast<const uint4*>(tab + (size_t)(2 * rp + par) * kpad + jl)
                   : make_uint4(0, 0, 0, 0);
      }
    };
    load_chunk(0);
    for (int k0 = 0; k0 < npar; k0 += 32) {
      __builtin_amdgcn_wave_barrier();  // the previous chunk's operand reads come first
#pragma unroll
      for (int u = 0; u < 32 / RPL; ++u) {
        unsigned* d = reinterpret_cast<unsigned*>(tw + (size_t)(u * RPL + lane / LPR) * TW + (lane % LPR) * EPL);
        d[0] = v[u].x;
        d[1] = v[u].y;
        d[2] = v[u].z;
        d[3] = v[u].w;
      }
      __builtin_amdgcn_wave_barrier();
      if (k0 + 32 < npar) load_chunk(k0 + 32);
#pragma unroll
      for (int s = 0; s < 32 / KS; ++s)
#pragma unroll
        for (int q = 0; q < QT; ++q) {
          // A[j][k] = P[row k0 + KS s + KV lg + e][latitude 16 (QT jq + q) + li]
          TT a[KV];
#pragma unroll
          for (int e = 0; e < KV; ++e) a[e] = tw[(size_t)(KS * s + KV * lg + e) * TW + 16 * q + li];
#pragma unroll
          for (int c = 0; c < NT; ++c) {
            const TT* bp = bs + ((size_t)par * NS + srow(c * 16 + li)) * bs_ld + k0 + KS * s + lg * KV;
            acc[q][c] = MT::mma(a, bp, acc[q][c]);
          }
        }
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      const int col = c0 + c * 16 + li;
      if (col >= ncol) continue;
      cpx<T>* dst = A.spec + A.items[A.item0 + (col >> 1)].soff + (size_t)m * h * 2 + par;
#pragma unroll
      for (int q = 0; q < QT; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = 16 * (QT * jq + q) + lg * 4 + i;
          if (j < h) reinterpret_cast<T*>(&dst[2 * j])[col & 1] = (T)acc[q][c][i];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// Single-item table Legendre stage of a heat apply on the vector units.  For
// one item the contractions are matrix-vector products bound by the table
// stream, so each table element is read once and used for both:
//   analysis   f_r = sum_j P_r(x_j) y_j     lane partials over the lane's 8
//              latitudes, then a reduction across the wave (permlane swaps
//              for lane bits 5 and 4, DPP for bits 3 .. 0) that leaves row
//              tile value k = 2 rr + c in the 32 / RT lanes from 32 k / RT
//   b_r = h_l f_r, passed to the wave's lanes through LDS
//   synthesis  G_j += P_r(x_j) b_r          the lane's own latitudes
// One workgroup of NW waves per order m; wave w takes rows of parity w & 1,
// RT at a time, lane L latitudes 8L .. 8L+7 (16-byte loads of the row-major
// table).  Loading the next tile ahead of the current one's use measured
// slower (a second tile of registers halves the resident waves).
// The waves' partial G of one parity are added in LDS in wave order.
// ---------------------------------------------------------------------------
template <typename TT>
struct GemvRow;
template <>
struct GemvRow<unsigned short> {  // 8 bfloat16 latitudes in one 16-byte load
  uint4 v;
  __device__ void load(const unsigned short* p, bool ok) {
    v = ok ? *reinterpret_cast<const uint4*>(p) : make_uint4(0, 0, 0, 0);
  }
  __device__ float operator[](int e) const {
    const unsigned w = e < 2 ? v.x : e < 4 ? v.y : e < 6 ? v.z : v.w;
    return __uint_as_float((e & 1) ? (w & 0xffff0000u) : (w << 16));
  }
};
template <>
struct GemvRow<float> {  // 8 float latitudes in two 16-byte loads
  float4 a, b;
  __device__ void load(const float* p, bool ok) {
    a = ok ? reinterpret_cast<const float4*>(p)[0] : make_float4(0.f, 0.f, 0.f, 0.f);
    b = ok ? reinterpret_cast<const float4*>(p)[1] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __device__ float operator[](int e) const {
    const float4& q = e < 4 ? a : b;
    const int i = e & 3;
    return i == 0 ? q.x : i == 1 ? q.y : i == 2 ? q.z : q.w;
  }
};

// Launch shape: eight waves per order, tiles of four rows.  At 721x1440 (bf16
// table, one item, interleaved runs) 8 x 4 took 39.8 us per heat apply; 8 x 8
// 48 us (more registers: one workgroup per compute unit); 4 x 8 43 us; 4 x 4
// 56 us.
__host__ __device__ constexpr int gemv_waves() { return 8; }
__host__ __device__ constexpr int gemv_rows() { return 4; }
size_t gemv_lds_bytes() { return (size_t)gemv_waves() * (16 + 512 * 2) * sizeof(float); }

template <typename T, typename TT, int NW, int RT>
__global__ void __launch_bounds__(64 * NW) legendre_gemv_kernel(LegArgs<T> A) {
  static_assert(RT == 4 || RT == 8, "tiles of 4 or 8 rows");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* bw_all = reinterpret_cast<float*>(smem_raw);  // [NW][16] b of the wave's current tile
  float* gs = bw_all + NW * 16;                         // [NW][512][2] partial G
  const int L = A.L, h = A.h, kpad = A.hpad;
  const int m = A.morder ? A.morder[blockIdx.x] : (int)blockIdx.x, nr = L - m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int par = wave & 1, npar = (nr + 1 - par) / 2;
  const TT* tab = static_cast<const TT*>(A.tab) + tri_off(m, L) * kpad;
  const int j0 = 8 * lane;
  const bool lok = j0 < kpad;  // kpad is a multiple of 32: whole 8-latitude runs
  const ItemDev& it = A.items[A.item0];
  const cpx<T>* sp = A.spec + it.soff + (size_t)m * h * 2 + par;
  const T* hl = A.hl + (size_t)A.item0 * A.hl_stride + m;
  float yr[8], yi[8], gr[8], gi[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int j = j0 + e;
    cpx<T> y{0, 0};
    if (j < h) y = sp[2 * j];
    yr[e] = (float)y.x;
    yi[e] = (float)y.y;
    gr[e] = gi[e] = 0.f;
  }
  float* bw = bw_all + wave * 16;
  auto load_tile = [&](GemvRow<TT> (&P)[RT], int t) {
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      const int rp = t * RT + rr;
      P[rr].load(tab + (size_t)(2 * rp + par) * kpad + j0, lok && rp < npar);
    }
  };
  GemvRow<TT> P[RT];
  for (int t = wave >> 1; t * RT < npar; t += NW / 2) {
    load_tile(P, t);
    // lane partials: value k = 2 rr + c
    float v[2 * RT];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float pv = P[rr][e];
        sr = fmaf(pv, yr[e], sr);
        si = fmaf(pv, yi[e], si);
      }
      v[2 * rr] = sr;
      v[2 * rr + 1] = si;
    }
    // reduction across the wave, halving the values at each lane bit from 5
    // down until one value is left per lane, then summing over the rest
    float w[RT], x[RT / 2], y2[RT / 4];
#pragma unroll
    for (int k = 0; k < RT; ++k) w[k] = swap_add32(v[k], v[k + RT]);
#pragma unroll
    for (int k = 0; k < RT / 2; ++k) x[k] = swap_add16(w[k], w[k + RT / 2]);
    const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int k = 0; k < RT / 4; ++k) y2[k] = (b3 ? x[k + RT / 4] : x[k]) + dpp_f(b3 ? x[k] : x[k + RT / 4], 0);
    float z;
    if constexpr (RT == 8) {
      z = (b2 ? y2[1] : y2[0]) + dpp_f(b2 ? y2[0] : y2[1], 1);
    } else {
      z = y2[0] + dpp_f(y2[0], 1);
    }
    z += dpp_f(z, 2);
    z += dpp_f(z, 3);
    // b = h_l f for value k = lane / (32 / RT) (row 2 (RT t + k / 2) + par of the order)
    constexpr int SHV = RT == 8 ? 2 : 3;
    if ((lane & ((1 << SHV) - 1)) == 0) {
      const int k = lane >> SHV, rp = t * RT + (k >> 1);
      bw[k] = rp < npar ? z * (float)hl[2 * rp + par] : 0.f;
    }
    __builtin_amdgcn_wave_barrier();
    float b[2 * RT];
#pragma unroll
    for (int q = 0; q < RT / 2; ++q) {
      const float4 b4 = reinterpret_cast<const float4*>(bw)[q];
      b[4 * q] = b4.x;
      b[4 * q + 1] = b4.y;
      b[4 * q + 2] = b4.z;
      b[4 * q + 3] = b4.w;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float pv = P[rr][e];
        gr[e] = fmaf(pv, b[2 * rr], gr[e]);
        gi[e] = fmaf(pv, b[2 * rr + 1], gi[e]);
      }
  }
  // partial G of this wave, then the sum over the waves of each parity
  if (lok) {
    float4* g4 = reinterpret_cast<float4*>(gs + ((size_t)wave * 512 + j0) * 2);
#pragma unroll
    for (int q = 0; q < 4; ++q) g4[q] = make_float4(gr[2 * q], gi[2 * q], gr[2 * q + 1], gi[2 * q + 1]);
  }
  __syncthreads();
  cpx<T>* out = A.spec + it.soff + (size_t)m * h * 2;
  for (int idx = tid; idx < 2 * h; idx += 64 * NW) {
    const int pp = idx >= h ? 1 : 0, j = idx - pp * h;
    float sr = 0.f, si = 0.f;
    for (int w2 = pp; w2 < NW; w2 += 2) {
      const float2 g = reinterpret_cast<const float2*>(gs)[(size_t)w2 * 512 + j];
      sr += g.x;
      si += g.y;
    }
    out[2 * j + pp] = cpx<T>{(T)sr, (T)si};
  }
}

// ---------------------------------------------------------------------------
// Recurrence-fed matrix-core Legendre kernel (float32 fields, batches).
//
// P̄_l^m is generated by the float64 three-term recurrence (as in the VALU
// kernels) and contracted on matrix cores against all the items of a column
// chunk at once, so one recurrence serves 8 NT items instead of one or two.
// One workgroup per (order m, chunk of 8 NT items = 16 NT real columns); its
// NW = ceil(h / 64) waves split the latitudes, each lane running the chain of
// one latitude j.  Rows are taken in blocks of 32 (16 per parity), rows of
// one parity forming the M (analysis) or K (synthesis) dimension of a tile:
//   analysis   D[r][n] = sum_j R_r(x_j) Y[j][n]     K = the wave's 64 latitudes
//   combine    b[r][n] = gamma_r^2 h_l(item) sum over waves of D (fixed order)
//   synthesis  G[j][n] = sum_r R_r(x_j) b[r][n]     K = rows of one parity
// (P̄ = gamma R; the folded spectrum entries E/O are the columns n of one
// parity).  The analysis A operand needs the recurrence values with the
// latitude along K, so each block's values pass through a per-wave LDS tile;
// the synthesis A operand has the rows along K, which a lane already holds,
// and a 4 x 4 exchange of lane groups (permlane swaps) puts them in operand
// order.  Operands: float32 (v_mfma_f32_16x16x4_f32), bfloat16
// (v_mfma_f32_16x16x16_bf16) or split bfloat16 (x = hi + lo, two bf16 with
// round-to-nearest; products hi*hi + hi*lo + lo*hi, three MFMAs): relative
// error about 2^-16 per product instead of 2^-8.  Accumulation is float32.
// ---------------------------------------------------------------------------
typedef short rm_short4 __attribute__((ext_vector_type(4)));

// bf16 bits of v, round to nearest even (the hardware conversion)
__device__ __forceinline__ unsigned rm_bf16(float v) {
  return (unsigned)__builtin_bit_cast(unsigned short, (__bf16)v);
}

template <int OP>
struct RmTraits;
template <>
struct RmTraits<RM_F32> {
  static constexpr int KS = 4;       // k per MFMA
  static constexpr int PLANES = 1;   // LDS planes (hi, lo)
  static constexpr int ES = 4;       // bytes per element of a plane
  struct Op { float v; };
  __device__ static void put(unsigned char* base, size_t plane, size_t idx, float v) {
    reinterpret_cast<float*>(base)[idx] = v;
  }
  // k-run of one lane from a plane row (KS / 4 groups of 4... one value for f32)
  __device__ static Op get(const unsigned char* base, size_t plane, size_t idx) {
    return {reinterpret_cast<const float*>(base)[idx]};
  }
  __device__ static f32x4_t mma(const Op& a, const Op& b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v, b.v, c, 0, 0, 0);
  }
  __device__ static Op make(const float (&x)[1]) { return {x[0]}; }
  // four consecutive elements, idx a multiple of 2
  __device__ static void put4(unsigned char* base, size_t plane, size_t idx, const float (&v)[4]) {
    float2* p = reinterpret_cast<float2*>(reinterpret_cast<float*>(base) + idx);
    p[0] = make_float2(v[0], v[1]);
    p[1] = make_float2(v[2], v[3]);
  }
};
template <>
struct RmTraits<RM_BF16> {
  static constexpr int KS = 16;
  static constexpr int PLANES = 1;
  static constexpr int ES = 2;
  struct Op { uint2 h; };
  __device__ static void put(unsigned char* base, size_t plane, size_t idx, float v) {
    reinterpret_cast<unsigned short*>(base)[idx] = (unsigned short)rm_bf16(v);
  }
  __device__ static Op get(const unsigned char* base, size_t plane, size_t idx) {
    return {*reinterpret_cast<const uint2*>(reinterpret_cast<const unsigned short*>(base) + idx)};
  }
  __device__ static f32x4_t mma(const Op& a, const Op& b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(rm_short4, a.h),
                                                     __builtin_bit_cast(rm_short4, b.h), c, 0, 0, 0);
  }
  __device__ static Op make(const float (&x)[4]) {
    return {make_uint2(rm_bf16(x[0]) | (rm_bf16(x[1]) << 16), rm_bf16(x[2]) | (rm_bf16(x[3]) << 16))};
  }
  // four consecutive elements, idx a multiple of 4
  __device__ static void put4(unsigned char* base, size_t plane, size_t idx, const float (&v)[4]) {
    *reinterpret_cast<uint2*>(reinterpret_cast<unsigned short*>(base) + idx) = make(v).h;
  }
};
template <>
struct RmTraits<RM_BF16X3> {
  static constexpr int KS = 16;
  static constexpr int PLANES = 2;
  static constexpr int ES = 2;
  struct Op { uint2 h, l; };
  __device__ static void put(unsigned char* base, size_t plane, size_t idx, float v) {
    const unsigned hb = rm_bf16(v);
    const float lo = v - __uint_as_float(hb << 16);
    unsigned short* p = reinterpret_cast<unsigned short*>(base);
    p[idx] = (unsigned short)hb;
    p[plane + idx] = (unsigned short)rm_bf16(lo);
  }
  __device__ static Op get(const unsigned char* base, size_t plane, size_t idx) {
    const unsigned short* p = reinterpret_cast<const unsigned short*>(base);
    return {*reinterpret_cast<const uint2*>(p + idx), *reinterpret_cast<const uint2*>(p + plane + idx)};
  }
  __device__ static f32x4_t mma(const Op& a, const Op& b, f32x4_t c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(rm_short4, a.l),
                                                  __builtin_bit_cast(rm_short4, b.h), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(rm_short4, a.h),
                                                  __builtin_bit_cast(rm_short4, b.l), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(rm_short4, a.h),
                                                     __builtin_bit_cast(rm_short4, b.h), c, 0, 0, 0);
  }
  __device__ static Op make(const float (&x)[4]) {
    unsigned hb[4], lb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      hb[e] = rm_bf16(x[e]);
      lb[e] = rm_bf16(x[e] - __uint_as_float(hb[e] << 16));
    }
    return {make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16)),
            make_uint2(lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16))};
  }
  // four consecutive elements, idx a multiple of 4
  __device__ static void put4(unsigned char* base, size_t plane, size_t idx, const float (&v)[4]) {
    const Op o = make(v);
    unsigned short* p = reinterpret_cast<unsigned short*>(base);
    *reinterpret_cast<uint2*>(p + idx) = o.h;
    *reinterpret_cast<uint2*>(p + plane + idx) = o.l;
  }
};

// float value of a float64 recurrence term, kept opaque so that a later
// rounding to bfloat16 stays a float -> bfloat16 conversion (fused with the
// float64 -> float one, the compiler emits an exact double -> bfloat16
// conversion costing several instructions per value)
__device__ __forceinline__ float rm_f32(double x) {
  float f = (float)x;
  asm("" : "+v"(f));
  return f;
}

// 4 x 4 exchange of lane groups: afterwards register t holds, in lane group g,
// what lane group t held in register g (lane groups = 16-lane rows).
__device__ __forceinline__ void lanegroup_transpose4(unsigned& r0, unsigned& r1, unsigned& r2, unsigned& r3) {
  auto a = __builtin_amdgcn_permlane32_swap(r0, r2, false, false);
  auto b = __builtin_amdgcn_permlane32_swap(r1, r3, false, false);
  auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
  auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
  r0 = c[0];
  r1 = c[1];
  r2 = d[0];
  r3 = d[1];
}

// LDS layout of legendre_rmma_kernel (bytes), shared with the host.
struct RmLayout {
  int nb, ncol, pld, bld;
  size_t o_p, o_d, o_b, o_c, o_s, total, pplane, bplane;
};
__host__ __device__ inline RmLayout rm_layout(int L, int h, int nt, int nw, int es, int planes) {
  RmLayout q;
  q.nb = (L + 31) / 32;              // row blocks of the longest order
  q.ncol = 16 * nt;
  // row pitches (elements): float rows odd, so the lanes of a k-slice read
  // distinct banks; bfloat16 rows keep 8-byte operand reads aligned.  b holds
  // one block's 16 rows per parity: a pitch of 18 floats puts the 32 lanes of
  // a half-wave's k-slice on distinct banks
  q.pld = es == 4 ? 65 : 68;
  q.bld = es == 4 ? 18 : 20;
  q.pplane = (size_t)nw * 32 * q.pld;
  q.bplane = (size_t)2 * q.ncol * q.bld;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 15) / 16 * 16; return o; };
  q.o_p = take(q.pplane * planes * es);
  q.o_d = take(sizeof(float) * nw * 2 * q.ncol * 20);
  q.o_b = take(q.bplane * planes * es);
  q.o_c = take(sizeof(double) * (32 * q.nb + 1));
  q.o_s = take(sizeof(double) * 2 * 8 * nt * 16);  // the block's gamma^2 h_l per parity, item, row
  q.total = off;
  return q;
}

// Split bfloat16 with 8 items per group is held to three waves per SIMD (at
// most 168 registers); the other forms reach it or exceed it by design.
template <typename T, int OP, int NT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu((OP == RM_BF16X3 && NT == 1) ? 3 : 1)))
legendre_rmma_kernel(LegArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using TR = RmTraits<OP>;
  using Op = typename TR::Op;
  constexpr int KS = TR::KS, ES = TR::ES, PL = TR::PLANES;
  constexpr int NKS = 64 / KS;        // k steps over a wave's 64 latitudes
  constexpr int RQ = OP == RM_BF16X3 ? 8 : 16;  // recurrence coefficients held in registers at once
  const int L = A.L, h = A.h;
  const int nw = blockDim.x >> 6;
  const RmLayout Q = rm_layout(L, h, NT, nw, ES, PL);
  // workgroups are dispatched in linear order: take orders longest first, all
  // column chunks of an order together
  const int lin = blockIdx.x + gridDim.x * blockIdx.y;
  const int m = lin / gridDim.y;
  const int nr = L - m;
  const int nblk = (nr + 31) / 32;
  const int c0 = (lin - m * gridDim.y) * Q.ncol;
  const int ncol = 2 * A.nb;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lg = lane >> 4;
  unsigned char* Pt = smem_raw + Q.o_p + (size_t)wave * 32 * Q.pld * ES;
  float* Dp = reinterpret_cast<float*>(smem_raw + Q.o_d);
  unsigned char* Bs = smem_raw + Q.o_b;
  double* cf = reinterpret_cast<double*>(smem_raw + Q.o_c);
  const long long toff = tri_off(m, L);
  const int nit = min(8 * NT, A.nb - c0 / 2);                 // items of this chunk
  const int ncomb = 2 * 16 * Q.ncol;                           // combine elements per block
  double* scd = reinterpret_cast<double*>(smem_raw + Q.o_s);  // [parity][8 NT items][16 rows] gamma^2 h_l
  // items of one launch group are consecutive in the workspace, each holding
  // 2 L h complex spectral entries: this chunk's spectra start here
  const float4* spc = reinterpret_cast<const float4*>(A.spec + A.soff0) + (size_t)(c0 / 2) * L * h + (size_t)m * h;
  const int j = 64 * wave + lane;
  const double xj = A.xs[min(j, h - 1)];
  const double sd = A.rseed[(size_t)m * h + min(j, h - 1)];

  // This wave's latitudes of the items' folded spectra, the analysis B
  // operands, loaded straight into registers (k = latitude 64 wave + KS s + the
  // lane group's k-run).  Each lane needs one component of an item's (E, O)
  // pair per latitude; the two lanes of an item (real / imaginary column)
  // each load whole 16-byte pairs of alternate latitudes and trade halves by
  // DPP.  The loads are issued first, then the order's recurrence
  // coefficients (zero past its end) are staged for the whole workgroup.
  constexpr int NE = KS == 4 ? 1 : 4;         // latitudes per k step and lane
  constexpr int NG = NKS * NE / 2;            // latitude pairs per lane and item
  const bool odd = li & 1;
  // latitude of pair g for the even (q = 0) or odd (q = 1) lane
  auto pair_lat = [&](int g, int q) {
    const int s = KS == 4 ? 2 * g + q : g >> 1, e = KS == 4 ? 0 : 2 * (g & 1) + q;
    return 64 * wave + KS * s + (KS == 4 ? lg : 4 * lg + e);
  };
  float4 fl[NT][NG];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int il = 8 * t + (li >> 1);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int jj = pair_lat(g, odd ? 1 : 0);
      fl[t][g] = il < nit && jj < h ? spc[(size_t)il * L * h + jj] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  {
    double cv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) cv[u] = A.rcoef[toff + min(tid + u * (int)blockDim.x, nr - 1)];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = tid + u * (int)blockDim.x;
      if (r <= 32 * nblk) cf[r] = (r < nr && r > 0) ? cv[u] : 0.0;
    }
    for (int r = tid + 2 * blockDim.x; r <= 32 * nblk; r += blockDim.x)
      cf[r] = (r < nr && r > 0) ? A.rcoef[toff + min(r, nr - 1)] : 0.0;
  }
  const double seed = j < h ? sd : 0.0;   // lanes past the last latitude run a zero chain
  Op yb[NKS][2][NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    float xv[NKS][2][NE];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const float4 F = fl[t][g];
      // the even lane sends (E im, O im) of its latitude, the odd lane (E re,
      // O re) of its own; each keeps its component of both latitudes
      const float r0 = dpp_f(odd ? F.x : F.y, 3), r1 = dpp_f(odd ? F.z : F.w, 3);
      const float a0 = odd ? r0 : F.x, a1 = odd ? r1 : F.z;   // the even lane's latitude
      const float b0 = odd ? F.y : r0, b1 = odd ? F.w : r1;   // the odd lane's latitude
      const int sa = KS == 4 ? 2 * g : g >> 1, ea = KS == 4 ? 0 : 2 * (g & 1);
      const int sb = KS == 4 ? 2 * g + 1 : g >> 1, eb = KS == 4 ? 0 : 2 * (g & 1) + 1;
      xv[sa][0][ea] = a0;
      xv[sa][1][ea] = a1;
      xv[sb][0][eb] = b0;
      xv[sb][1][eb] = b1;
    }
#pragma unroll
    for (int s = 0; s < NKS; ++s)
#pragma unroll
      for (int par = 0; par < 2; ++par) yb[s][par][t] = TR::make(xv[s][par]);
  }
  __syncthreads();  // the coefficients are staged

  // ---- one pass over the order's rows, 32 at a time: the block's analysis
  // f = sum_j P y (partials of the waves combined in LDS), b = gamma^2 h_l f,
  // then the block's synthesis term G += sum_l P b from the same recurrence
  // values (kept in registers; lane-group exchanges put them in operand order)
  f32x4_t G[2][4][NT];
#pragma unroll
  for (int par = 0; par < 2; ++par)
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int t = 0; t < NT; ++t) G[par][jt][t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  double R1 = seed, R2 = 0.0;
  for (int blk = 0; blk < nblk; ++blk) {
    const int r0 = 32 * blk;
    // gamma and h_l of this block's rows, loaded now, stored to LDS before the
    // barrier, used by the combine after it
    const int gr = min(r0 + (tid & 31), nr - 1);
    const double gld = A.rgam[toff + gr];
    float hld[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = min(tid + u * (int)blockDim.x, 8 * NT * 32 - 1), i = min(e >> 5, nit - 1);
      hld[u] = A.hl[(size_t)(A.item0 + c0 / 2 + i) * A.hl_stride + m + min(r0 + (e & 31), nr - 1)];
    }
    float v[32];
#pragma unroll
    for (int hq = 0; hq < 32; hq += RQ) {  // coefficients in batches of RQ (registers)
      double cq[RQ];
#pragma unroll
      for (int q = 0; q < RQ; ++q) cq[q] = cf[r0 + hq + q + 1];
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        v[hq + q] = rm_f32(R1);
        if constexpr (OP == RM_F32) TR::put(Pt, Q.pplane, (size_t)(hq + q) * Q.pld + lane, v[hq + q]);
        const double rn = fma(cq[q] * xj, R1, R2);
        R2 = R1;
        R1 = rn;
      }
    }
    // bfloat16 forms: the block's values rounded once, packed two rows of a
    // parity per word (rows 2(4u+2w)+par and the next of that parity), used by
    // the synthesis operands and written to the tile as 16-bit halves; tile
    // rows are stored by parity (row 2k+par at 16 par + k), so that the 16
    // lanes of an 8-byte operand read fall on distinct banks
    unsigned hwp[2][2][4], lwp[2][2][4];
    if constexpr (OP != RM_F32) {
      unsigned short* th = reinterpret_cast<unsigned short*>(Pt);
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w2 = 0; w2 < 2; ++w2) {
            const float x0 = v[2 * (4 * u + 2 * w2) + par], x1 = v[2 * (4 * u + 2 * w2 + 1) + par];
            const unsigned h0 = rm_bf16(x0), h1 = rm_bf16(x1);
            hwp[par][w2][u] = h0 | (h1 << 16);
            const size_t ra = (size_t)(16 * par + 4 * u + 2 * w2) * Q.pld + lane;
            th[ra] = (unsigned short)h0;
            th[ra + Q.pld] = (unsigned short)h1;
            if constexpr (OP == RM_BF16X3) {
              const unsigned l0 = rm_bf16(x0 - __uint_as_float(h0 << 16));
              const unsigned l1 = rm_bf16(x1 - __uint_as_float(h1 << 16));
              lwp[par][w2][u] = l0 | (l1 << 16);
              th[Q.pplane + ra] = (unsigned short)l0;
              th[Q.pplane + ra + Q.pld] = (unsigned short)l1;
            }
          }
    }
    f32x4_t acc[2][NT];
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[par][t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        // A[i][k] = R_{r0 + 2i + par}(x_{64 wave + KS s + k})
        const int kk = KS * s + (KS == 4 ? lg : 4 * lg);
        const int trow = OP == RM_F32 ? 2 * li + par : 16 * par + li;
        const Op a = TR::get(Pt, Q.pplane, (size_t)trow * Q.pld + kk);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[par][t] = TR::mma(a, yb[s][par][t], acc[par][t]);
      }
    }
    // the combine's scale gamma^2 h_l per (parity, item, row of the parity);
    // zero past the order's end and past the chunk's items (blockDim is a
    // multiple of 32, so e & 31 is this thread's gamma row)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + u * (int)blockDim.x, i = e >> 5, rr = e & 31;
      if (e < 8 * NT * 32) {
        const double g = r0 + rr < nr && i < nit ? gld : 0.0;
        scd[((rr & 1) * 8 * NT + i) * 16 + (rr >> 1)] = g * g * (double)hld[u];
      }
    }
    for (int e = tid + 2 * blockDim.x; e < 8 * NT * 32; e += blockDim.x) {  // one-wave workgroups of 16 items
      const int i = e >> 5, rr = e & 31, r = r0 + rr;
      const bool ok = r < nr && i < nit;
      const double g = ok ? A.rgam[toff + r] : 0.0;
      const float hv = ok ? (float)A.hl[(size_t)(A.item0 + c0 / 2 + i) * A.hl_stride + m + r] : 0.f;
      scd[((rr & 1) * 8 * NT + i) * 16 + (rr >> 1)] = g * g * (double)hv;
    }
    // wave partials, [wave][parity][column][row of the parity] (rows padded to 20)
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        *reinterpret_cast<f32x4_t*>(Dp + (((size_t)wave * 2 + par) * Q.ncol + 16 * t + li) * 20 + 4 * lg) =
            acc[par][t];
    __syncthreads();
    // b = gamma^2 h_l (sum over the waves), in the operand format, rows of one
    // parity contiguous, four rows per thread; rows past the order's end are
    // zero (their scale is zero)
    for (int idx = tid; idx < ncomb / 4; idx += blockDim.x) {
      constexpr int NC = 16 * NT;
      const int pn = idx >> 2, q4 = idx & 3;
      const int par = pn >= NC ? 1 : 0, n = pn - par * NC;
      const f32x4_t* dp = reinterpret_cast<const f32x4_t*>(Dp) + (par * NC + n) * 5 + q4;
      f32x4_t sum = f32x4_t{0.f, 0.f, 0.f, 0.f};
      for (int w = 0; w < nw; ++w) sum += dp[w * 2 * NC * 5];
      const double* sc = scd + (par * 8 * NT + (n >> 1)) * 16 + 4 * q4;
      float o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = (float)((double)sum[e] * sc[e]);
      TR::put4(Bs, Q.bplane, (size_t)(par * NC + n) * Q.bld + 4 * q4, o);
    }
    __syncthreads();
    // the block's synthesis term
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      if constexpr (OP == RM_F32) {
        // K step s: rows of this parity 4s .. 4s+3 of the block
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          unsigned a[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) a[e] = __float_as_uint(v[2 * (4 * s + e) + par]);
          lanegroup_transpose4(a[0], a[1], a[2], a[3]);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const Op b = TR::get(Bs, Q.bplane, ((size_t)par * Q.ncol + 16 * t + li) * Q.bld + 4 * s + lg);
#pragma unroll
            for (int jt = 0; jt < 4; ++jt) G[par][jt][t] = TR::mma(Op{__uint_as_float(a[jt])}, b, G[par][jt][t]);
          }
        }
      } else {
        // one K step: the 16 rows of this parity; lane group g holds rows 4g .. 4g+3
        unsigned hw[2][4], lw[2][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w2 = 0; w2 < 2; ++w2) {
            hw[w2][u] = hwp[par][w2][u];
            if constexpr (OP == RM_BF16X3) lw[w2][u] = lwp[par][w2][u];
          }
#pragma unroll
        for (int w2 = 0; w2 < 2; ++w2) {
          lanegroup_transpose4(hw[w2][0], hw[w2][1], hw[w2][2], hw[w2][3]);
          if constexpr (OP == RM_BF16X3) lanegroup_transpose4(lw[w2][0], lw[w2][1], lw[w2][2], lw[w2][3]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const Op b = TR::get(Bs, Q.bplane, ((size_t)par * Q.ncol + 16 * t + li) * Q.bld + 4 * lg);
#pragma unroll
          for (int jt = 0; jt < 4; ++jt) {
            Op a;
            a.h = make_uint2(hw[0][jt], hw[1][jt]);
            if constexpr (OP == RM_BF16X3) a.l = make_uint2(lw[0][jt], lw[1][jt]);
            G[par][jt][t] = TR::mma(a, b, G[par][jt][t]);
          }
        }
      }
    }
  }
  // ---- the order's folded spectrum: G[j][n] (j = 64 wave + 16 jt + 4 lg + e)
  // stored straight from the accumulators: the two lanes of an item (its real
  // and imaginary column) trade halves so that each writes whole (E, O)
  // complex pairs, 16 bytes per latitude (gathering through LDS first, for
  // fully contiguous stores, measured 3 % slower)
  float4* dsc = reinterpret_cast<float4*>(A.spec + A.soff0) + (size_t)(c0 / 2) * L * h + (size_t)m * h;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int il = 8 * t + (li >> 1);
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int ep = 0; ep < 2; ++ep) {
        // the even lane writes latitude e = 2 ep, the odd lane e = 2 ep + 1
        const int ea = 2 * ep, eb = 2 * ep + 1;
        const float r0 = dpp_f(odd ? G[0][jt][t][ea] : G[0][jt][t][eb], 3);
        const float r1 = dpp_f(odd ? G[1][jt][t][ea] : G[1][jt][t][eb], 3);
        const float4 o = odd ? make_float4(r0, G[0][jt][t][eb], r1, G[1][jt][t][eb])
                             : make_float4(G[0][jt][t][ea], r0, G[1][jt][t][ea], r1);
        const int jj = 64 * wave + 16 * jt + 4 * lg + (odd ? eb : ea);
        if (il < nit && jj < h) dsc[(size_t)il * L * h + jj] = o;
      }
  }
}

// ---------------------------------------------------------------------------
// Per-item final reductions: cost, e_marg history and final residual, masses.
// res[item*8 + .] = {cost, err, m(p), m(q), ||p||, 0, 0, 0}.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) reduce_kernel(RowArgs<T> A, int nchk_done, double* res, double* ehist) {
  __shared__ double sh[16];
  const int it = A.item0 + blockIdx.x;
  const int h = A.h;
  double s[4] = {0, 0, 0, 0};
  for (int q = threadIdx.x; q < h; q += blockDim.x)
    for (int c = 0; c < 4; ++c) s[c] += A.prep[((size_t)it * A.hs + q) * 4 + c];
  for (int c = 0; c < 4; ++c) s[c] = block_sum(s[c], sh);
  const double pn = sqrt(s[0]);
  double fin = 0.0;
  if (A.chk_slot >= 0) {
    for (int q = threadIdx.x; q < h; q += blockDim.x) fin += A.rhist[((size_t)it * A.nslot + A.chk_slot) * A.hs + q];
    fin = block_sum(fin, sh);
  }
  // one wave per history slot (fixed summation order, no barriers)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wave; c < nchk_done; c += nw) {
    double e = 0.0;
    for (int q = lane; q < h; q += 64) e += A.rhist[((size_t)it * A.nslot + c) * A.hs + q];
    e = wave_sum(e);
    if (lane == 0) ehist[(size_t)it * A.nslot + c] = sqrt(e) / pn;
  }
  if (threadIdx.x == 0) {
    double* r = res + (size_t)it * 8;
    r[0] = s[3];
    r[1] = sqrt(fin) / pn;
    r[2] = s[1];
    r[3] = s[2];
    r[4] = pn;
  }
}

// ---------------------------------------------------------------------------
// Gauge of iteration k per item (g_k = s_k for balanced items), one block per item.
// ---------------------------------------------------------------------------
// (g_k, S_A, S_B) of iteration k per item, from the partial sums of its two halves.
template <typename T>
__global__ void __launch_bounds__(256) gauge3_kernel(RowArgs<T> A, int k, double* gout) {
  __shared__ double sh[16];
  const int it = A.item0 + blockIdx.x;
  const ItemDev I = A.items[it];
  const double* R = A.red + ((size_t)(k & 1) * A.nitems_all + it) * (size_t)A.hs * RED_SLOTS;
  double s0 = 0.0, s1 = 0.0;
  for (int q = threadIdx.x; q < A.h; q += blockDim.x) {
    s0 += R[(size_t)q * RED_SLOTS + 0];
    s1 += R[(size_t)q * RED_SLOTS + 1];
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    gout[3 * it] = I.balanced ? s0 : exp(-(0.5 * I.tau * (log(s0) - log(s1))) / I.eps);
    gout[3 * it + 1] = s0;
    gout[3 * it + 2] = s1;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) gauge_kernel(RowArgs<T> A, int k, double* gout) {
  __shared__ double sh[16];
  const int it = A.item0 + blockIdx.x;
  const ItemDev I = A.items[it];
  const double g = gauge(A, I, it, k, sh);
  if (threadIdx.x == 0) gout[it] = g;
}

// ---------------------------------------------------------------------------
// Row statistics of a gradient field for the regional attribution: per
// (row, item) the float64 sums sum a, sum a g and sum a g^2 of g = d / a over
// the row's points (d: the field, a: the point areas).  grid = (nlat, items).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) row_stats_kernel(RowArgs<T> A, const T* d, const long long* foff,
                                                        const double* aw, double* out) {
  __shared__ double sh[16];
  const int row = blockIdx.x, it = blockIdx.y;
  const int nlat = A.nlat;
  const int jp = row < A.h ? row : nlat - 1 - row;
  int len = A.nlon;
  long long start = (long long)row * A.nlon;
  if (A.ring) {
    len = A.ring[jp].len;
    start = row == jp ? A.ring[jp].off1 : A.ring[jp].off2;
  }
  const double a = aw[jp];  // double even for float fields: the statistic is taken in double
  const T* x = d + foff[it] + start;
  double s1 = 0.0, s2 = 0.0;
  for (int c = threadIdx.x; c < len; c += blockDim.x) {
    const double v = (double)x[c];
    s1 += v;           // a g = d
    s2 += v * v / a;   // a g^2 = d^2 / a
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    double* o = out + ((size_t)it * nlat + row) * 3;
    o[0] = a * len;
    o[1] = s1;
    o[2] = s2;
  }
}

template <typename T>
hipError_t launch_row_stats(const RowArgs<T>& a, int nitems, const T* d, const long long* foff, const double* aw,
                            double* out, hipStream_t stream) {
  hipLaunchKernelGGL(row_stats_kernel<T>, dim3(a.nlat, nitems), dim3(256), 0, stream, a, d, foff, aw, out);
  return hipGetLastError();
}
template hipError_t launch_row_stats<float>(const RowArgs<float>&, int, const float*, const long long*,
                                            const double*, double*, hipStream_t);
template hipError_t launch_row_stats<double>(const RowArgs<double>&, int, const double*, const long long*,
                                             const double*, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Per-pair gradient combination: out = wa (x1 - (x2 + x3)/2) + coef a.
// grid = (ceil(maxn / 256), npairs).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) combine_kernel(const CombineDev* __restrict__ D, T* out) {
  const CombineDev d = D[blockIdx.y];
  const long long n = d.n;
  const long long x = (long long)blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
  int jr = 0;
  if (!d.equal_area) {
    const int row = (int)(x / d.nlon);
    jr = row < d.h ? row : d.nlat - 1 - row;
  }
  const double a = (double)static_cast<const T*>(d.aw)[jr];
  const double v1 = (double)static_cast<const T*>(d.x1)[d.off1 + x];
  const double v2 = (double)static_cast<const T*>(d.x2)[d.off2 + x];
  const double v3 = (double)static_cast<const T*>(d.x3)[d.off3 + x];
  const double w = d.mul_area ? a : 1.0;
  out[d.off_out + x] = (T)(w * (v1 - 0.5 * (v2 + v3)) + d.coef * a);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Optional start/stop events of the next row or Legendre launch: the events
// are attached to the dispatch itself (hipExtLaunchKernelGGL), so they time
// the kernel's execution rather than the gap before it.
static thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

#define SHOT_LAUNCH(kernel, grid, block, lds, stream, ...)                                         \
  do {                                                                                             \
    if (g_ev_start && g_ev_stop) {                                                                 \
      hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, g_ev_start, g_ev_stop, 0, __VA_ARGS__); \
    } else {                                                                                       \
      hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                           \
    }                                                                                              \
    g_ev_start = g_ev_stop = nullptr;                                                              \
  } while (0)
// Row pairs per workgroup: the most (1, 2 or 4) whose two FFT buffers fit in
// LDS, with at most 1440 points of rows per group (192 items of 720-point
// rows: 250 us with 4 pairs per group, 226 us with 2), while the launch keeps
// at least ~2048 workgroups.
int row_pairs_per_group(int h, int nlon, int nb, size_t cs) {
  int rpw = 4;
  while (rpw > 1 && ((size_t)2 * rpw * nlon * cs > 60 * 1024 || rpw * nlon > 1440 ||
                     (long long)((h + rpw - 1) / rpw) * nb < 2048))
    rpw >>= 1;
  return rpw;
}

template <typename T, int RPW, int NC, int BS = 256>
static hipError_t launch_rows_nc(const RowArgs<T>& a, int nb, hipStream_t stream) {
  dim3 grid((a.h + RPW - 1) / RPW, nb);
  RowArgs<T> b = a;
  // two FFT buffers per pair plus the twiddles, in LDS (ring grids size them
  // by their longest ring or Bluestein convolution); beyond 64 KiB (fp64 rows
  // of 1440 or more points, long rings) the dynamic-LDS limit is raised, up
  // to 96 KiB for 2048-point fp64 rows and 160 KiB for rings
  const size_t nbuf = a.ring ? (size_t)a.nbuf : (size_t)a.nlon;
  const size_t lds = (size_t)(2 * RPW + 1) * nbuf * sizeof(cpx<T>);
  if (lds > 65536) {
    static size_t attr_bytes = 65536;  // dynamic LDS enabled so far, per kernel instantiation
    if (lds > attr_bytes) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&row_kernel<T, RPW, NC, BS>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr_bytes = lds;
    }
  }
  SHOT_LAUNCH((row_kernel<T, RPW, NC, BS>), grid, dim3(BS), lds, stream, b);
  return hipGetLastError();
}

// Transform lengths with a compile-time specialisation (the grids of the
// benchmarked workloads); any other length runs the runtime-length kernel.
template <typename T, int RPW>
static hipError_t launch_rows_rpw(const RowArgs<T>& a, int nb, hipStream_t stream) {
  if constexpr (sizeof(T) == 4) {
    switch (a.nlon) {
      case 180: return launch_rows_nc<T, RPW, 180>(a, nb, stream);
      case 360: return launch_rows_nc<T, RPW, 360>(a, nb, stream);
      case 720: return launch_rows_nc<T, RPW, 720>(a, nb, stream);
      case 1440: return launch_rows_nc<T, RPW, 1440>(a, nb, stream);
      default: break;
    }
  } else {
    if (a.nlon == 64) return launch_rows_nc<T, RPW, 64>(a, nb, stream);
  }
  return launch_rows_nc<T, RPW, 0>(a, nb, stream);
}

template <typename T, int RPW, int NC, int BS>
static hipError_t launch_sink(const RowArgs<T>& a, int nb, hipStream_t stream) {
  dim3 grid((a.h + RPW - 1) / RPW, nb);
  const size_t lds = (size_t)(2 * RPW + 1) * NC * sizeof(cpx<T>);
  SHOT_LAUNCH((row_sink_kernel<T, RPW, NC, BS>), grid, dim3(BS), lds, stream, a);
  return hipGetLastError();
}

template <typename T, int NC>
static hipError_t launch_sink_nc(const RowArgs<T>& a, int nb, hipStream_t stream) {
  const int rpw = row_pairs_per_group(a.h, a.nlon, nb, sizeof(cpx<T>));
  if ((size_t)(2 * rpw + 1) * NC * sizeof(cpx<T>) > 65536 - 1024) return hipErrorInvalidValue;
  if (rpw == 1) {
    // few row pairs: wider workgroups shorten each FFT stage
    if ((long long)a.h * nb < 1024) return launch_sink<T, 1, NC, 512>(a, nb, stream);
    return launch_sink<T, 1, NC, 256>(a, nb, stream);
  }
  if (rpw == 2) return launch_sink<T, 2, NC, 256>(a, nb, stream);
  return launch_sink<T, 4, NC, 256>(a, nb, stream);
}

template <typename T>
hipError_t launch_rows(const RowArgs<T>& a, int nb, hipStream_t stream) {
  // HEALPix: one ring pair per group; above Nside 64, rings of 4p pixels with
  // a large prime p make the generic-radix FFT stage the longest part of the
  // launch, so those groups get 1024 threads (512 in double precision, whose
  // registers would not fit 1024)
  if (a.ring && a.nlon > 256) {
    if constexpr (sizeof(T) == 4) return launch_rows_nc<T, 1, 0, 1024>(a, nb, stream);
    else return launch_rows_nc<T, 1, 0, 512>(a, nb, stream);
  }
  if (a.ring) return launch_rows_nc<T, 1, 0, 256>(a, nb, stream);
  if constexpr (sizeof(T) == 4) {
    if ((a.mode == ROW_SINK_U || a.mode == ROW_SINK_V) && a.tw) {
      switch (a.nlon) {
        case 180: return launch_sink_nc<T, 180>(a, nb, stream);
        case 360: return launch_sink_nc<T, 360>(a, nb, stream);
        case 720: return launch_sink_nc<T, 720>(a, nb, stream);
        case 1440: return launch_sink_nc<T, 1440>(a, nb, stream);
        default: break;
      }
    }
  }
  switch (row_pairs_per_group(a.h, a.nlon, nb, sizeof(cpx<T>))) {
    case 4: return launch_rows_rpw<T, 4>(a, nb, stream);
    case 2: return launch_rows_rpw<T, 2>(a, nb, stream);
    default: return launch_rows_rpw<T, 1>(a, nb, stream);
  }
}

template <typename T, typename TT, int IB>
static hipError_t launch_leg_ib(const LegArgs<T>& a, hipStream_t stream) {
  dim3 grid(a.L, (a.nb + IB - 1) / IB);
  const size_t lds = ((size_t)IB * 2 * a.h + (size_t)IB * a.L) * sizeof(cpx<T>);
  SHOT_LAUNCH((legendre_table_kernel<T, TT, IB>), grid, dim3(256), lds, stream, a);
  return hipGetLastError();
}

template <typename T, typename TT>
static hipError_t launch_leg_tt(const LegArgs<T>& a, int ib, hipStream_t stream) {
  switch (ib) {
    case 1: return launch_leg_ib<T, TT, 1>(a, stream);
    case 2: return launch_leg_ib<T, TT, 2>(a, stream);
    case 4: return launch_leg_ib<T, TT, 4>(a, stream);
    default: return launch_leg_ib<T, TT, 8>(a, stream);
  }
}

template <typename T, int IB, int JPT>
static hipError_t launch_recur(const LegArgs<T>& a, hipStream_t stream) {
  const int threads = ((a.h + JPT - 1) / JPT + 63) / 64 * 64;
  dim3 grid(a.L, (a.nb + IB - 1) / IB);
  const int npad = (a.L + 15) / 16 * 16;
  const size_t lds = (size_t)npad * 16 + (size_t)IB * npad * 16 + (size_t)2 * (threads / 64) * 32 * sizeof(T);
  SHOT_LAUNCH((legendre_recur_kernel<T, IB, JPT>), grid, dim3(threads), lds, stream, a);
  return hipGetLastError();
}

template <typename T, int IB>
static hipError_t launch_recur_ib(const LegArgs<T>& a, int jpt, hipStream_t stream) {
  switch (jpt) {
    case 1: return launch_recur<T, IB, 1>(a, stream);
    case 2: return launch_recur<T, IB, 2>(a, stream);
    default: return launch_recur<T, IB, 4>(a, stream);
  }
}

// Chains per thread for the recurrence kernel: the fewest that keep the
// block at <= 256 threads.
int recur_jpt(int h) { return h <= 256 ? 1 : (h <= 512 ? 2 : 4); }
int recur_jpt_valid(int h, int jpt) {
  return (jpt == 1 || jpt == 2 || jpt == 4) && (h + jpt - 1) / jpt <= 256;
}

template <typename T, int IB, int C>
static hipError_t launch_split(const LegArgs<T>& a, hipStream_t stream) {
  dim3 grid(a.nparts, (a.nb + IB - 1) / IB);
  const size_t lds = split_lds_bytes(a.maxlen, a.h, IB, (int)sizeof(T));
  SHOT_LAUNCH((legendre_split_kernel<T, IB, C, 32>), grid, dim3(256), lds, stream, a);
  return hipGetLastError();
}

template <typename T, int IB>
static hipError_t launch_split_ib(const LegArgs<T>& a, hipStream_t stream) {
  switch ((a.h + 63) / 64) {
    case 1: return launch_split<T, IB, 1>(a, stream);
    case 2: return launch_split<T, IB, 2>(a, stream);
    case 3: return launch_split<T, IB, 3>(a, stream);
    case 4: return launch_split<T, IB, 4>(a, stream);
    case 5: return launch_split<T, IB, 5>(a, stream);
    case 6: return launch_split<T, IB, 6>(a, stream);
    case 7: if constexpr (IB == 1) return launch_split<T, 1, 7>(a, stream); else return hipErrorInvalidValue;
    case 8: if constexpr (IB == 1) return launch_split<T, 1, 8>(a, stream); else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

size_t split_lds_bytes(int maxlen, int h, int ib, int real_bytes) {
  const size_t npad = (maxlen + 15) / 16 * 16 + 16;
  return npad * 16 + (size_t)ib * npad * 16 + (size_t)4 * ib * 2 * h * 2 * real_bytes;
}

template <typename T>
hipError_t launch_legendre_split(const LegArgs<T>& a, int ib, hipStream_t stream) {
  if (a.h > 512 || (ib >= 2 && a.h > 384)) return hipErrorInvalidValue;
  return ib >= 2 ? launch_split_ib<T, 2>(a, stream) : launch_split_ib<T, 1>(a, stream);
}
template hipError_t launch_legendre_split<float>(const LegArgs<float>&, int, hipStream_t);
template hipError_t launch_legendre_split<double>(const LegArgs<double>&, int, hipStream_t);

size_t mma_lds_bytes(int L, int hpad, int nt, int table_kind, bool narrow) {
  const int es = table_kind == TAB_BF16 ? 2 : 4;
  const int pad = table_kind == TAB_BF16 ? 8 : 1;
  const int NB = narrow ? 3 : 16 * nt, nw = mma_waves(narrow);
  return mma_tile_off(L, hpad, NB, es, pad) + (size_t)nw * 32 * mma_tile_ld(es, mma_tile_q(nw)) * es;
}

template <typename T, typename TT, int NT, bool NARROW>
static hipError_t launch_mma_nt(const LegArgs<T>& a, hipStream_t stream) {
  constexpr int NW = mma_waves(NARROW);
  dim3 grid(a.L, (2 * a.nb + 16 * NT - 1) / (16 * NT));
  const size_t lds = mma_lds_bytes(a.L, a.hpad, NT, sizeof(TT) == 2 ? TAB_BF16 : TAB_F32, NARROW);
  // The balanced order assumes the launch's workgroups sit three to a compute
  // unit in one column of tiles (one item of a bf16 table at L = 720: 3674 ->
  // 4094 iterations/s); with one workgroup per unit (fp32 tables of long
  // orders) or several column tiles it measured slower, so those run m = b.
  LegArgs<T> b = a;
  if (grid.y > 1 || lds > 160 * 1024 / 3) b.morder = nullptr;
  if (lds > 65536) {  // long orders of fp32 tables: one workgroup per compute unit
    static size_t attr_bytes = 65536;  // dynamic LDS enabled so far for this instantiation
    if (lds > attr_bytes) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&legendre_mma_kernel<T, TT, NT, NARROW, NW>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr_bytes = lds;
    }
  }
  SHOT_LAUNCH((legendre_mma_kernel<T, TT, NT, NARROW, NW>), grid, dim3(64 * NW), lds, stream, b);
  return hipGetLastError();
}

template <typename T, typename TT>
static hipError_t launch_mma_tt(const LegArgs<T>& a, int nt, hipStream_t stream) {
  switch (nt) {
    case 1:  // one item: its two columns only
      return a.nb == 1 ? launch_mma_nt<T, TT, 1, true>(a, stream) : launch_mma_nt<T, TT, 1, false>(a, stream);
    case 2: return launch_mma_nt<T, TT, 2, false>(a, stream);
    default: return launch_mma_nt<T, TT, 4, false>(a, stream);
  }
}

template <typename T>
hipError_t launch_legendre_mma(const LegArgs<T>& a, int table_kind, int nt, hipStream_t stream) {
  if (a.hpad % 32) return hipErrorInvalidValue;
  if (a.nb == 1 && a.mode == 0 && a.hpad <= 512) {  // one item: the vector-unit kernel
    const size_t lds = gemv_lds_bytes();
    if (table_kind == TAB_BF16)
      SHOT_LAUNCH((legendre_gemv_kernel<T, unsigned short, gemv_waves(), gemv_rows()>), dim3(a.L),
                  dim3(64 * gemv_waves()), lds, stream, a);
    else if (table_kind == TAB_F32)
      SHOT_LAUNCH((legendre_gemv_kernel<T, float, gemv_waves(), gemv_rows()>), dim3(a.L), dim3(64 * gemv_waves()),
                  lds, stream, a);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (table_kind == TAB_BF16) return launch_mma_tt<T, unsigned short>(a, nt, stream);
  if (table_kind == TAB_F32) return launch_mma_tt<T, float>(a, nt, stream);
  return hipErrorInvalidValue;
}
template hipError_t launch_legendre_mma<float>(const LegArgs<float>&, int, int, hipStream_t);
template hipError_t launch_legendre_mma<double>(const LegArgs<double>&, int, int, hipStream_t);

// Recurrence-fed matrix-core kernel: float32 fields only; waves = ceil(h/64) <= 8.
template <typename T, int OP, int NT>
static hipError_t launch_rmma_nt(const LegArgs<T>& a, hipStream_t stream) {
  if constexpr (sizeof(T) != 4) {
    return hipErrorInvalidValue;
  } else {
    using TR = RmTraits<OP>;
    const int nw = (a.h + 63) / 64;
    const RmLayout Q = rm_layout(a.L, a.h, NT, nw, TR::ES, TR::PLANES);
    if (nw > 8 || Q.total > 160 * 1024) return hipErrorInvalidValue;
    if (Q.total > 65536) {
      static size_t attr_bytes = 65536;  // dynamic LDS enabled so far for this instantiation
      if (Q.total > attr_bytes) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&legendre_rmma_kernel<T, OP, NT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)Q.total);
        if (e != hipSuccess) return e;
        attr_bytes = Q.total;
      }
    }
    dim3 grid(a.L, (2 * a.nb + Q.ncol - 1) / Q.ncol);
    SHOT_LAUNCH((legendre_rmma_kernel<T, OP, NT>), grid, dim3(64 * nw), Q.total, stream, a);
    return hipGetLastError();
  }
}

template <typename T, int OP>
static hipError_t launch_rmma_op(const LegArgs<T>& a, int nt, hipStream_t stream) {
  switch (nt) {
    case 1: return launch_rmma_nt<T, OP, 1>(a, stream);
    case 2: return launch_rmma_nt<T, OP, 2>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

size_t rmma_lds_bytes(int L, int h, int nt, int op) {
  const int nw = (h + 63) / 64;
  const int es = op == RM_F32 ? 4 : 2, planes = op == RM_BF16X3 ? 2 : 1;
  return rm_layout(L, h, nt, nw, es, planes).total;
}

template <typename T>
hipError_t launch_legendre_rmma(const LegArgs<T>& a, int op, int nt, hipStream_t stream) {
  switch (op) {
    case RM_F32: return launch_rmma_op<T, RM_F32>(a, nt, stream);
    case RM_BF16: return launch_rmma_op<T, RM_BF16>(a, nt, stream);
    case RM_BF16X3: return launch_rmma_op<T, RM_BF16X3>(a, nt, stream);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_legendre_rmma<float>(const LegArgs<float>&, int, int, hipStream_t);
template hipError_t launch_legendre_rmma<double>(const LegArgs<double>&, int, int, hipStream_t);

template <typename T>
hipError_t launch_legendre(const LegArgs<T>& a, int table_kind, int ib, hipStream_t stream) {
  switch (table_kind) {
    case TAB_F64: return launch_leg_tt<T, double>(a, ib, stream);
    case TAB_F32: return launch_leg_tt<T, float>(a, ib, stream);
    case TAB_BF16: return launch_leg_tt<T, unsigned short>(a, ib, stream);
    case TAB_RECUR: {
      if (a.h > 1024) return hipErrorInvalidValue;
      const int jpt = recur_jpt_valid(a.h, a.jpt) ? a.jpt : recur_jpt(a.h);
      switch (ib) {
        case 1: return launch_recur_ib<T, 1>(a, jpt, stream);
        case 2: return launch_recur_ib<T, 2>(a, jpt, stream);
        default: return launch_recur_ib<T, 4>(a, jpt, stream);
      }
    }
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_reduce(const RowArgs<T>& a, int nb, int nchk_done, double* res, double* ehist,
                         hipStream_t stream) {
  hipLaunchKernelGGL(reduce_kernel<T>, dim3(nb), dim3(256), 0, stream, a, nchk_done, res, ehist);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gauge3(const RowArgs<T>& a, int nb, int k, double* gout, hipStream_t stream) {
  hipLaunchKernelGGL(gauge3_kernel<T>, dim3(nb), dim3(256), 0, stream, a, k, gout);
  return hipGetLastError();
}
template hipError_t launch_gauge3<float>(const RowArgs<float>&, int, int, double*, hipStream_t);
template hipError_t launch_gauge3<double>(const RowArgs<double>&, int, int, double*, hipStream_t);

template <typename T>
hipError_t launch_gauge(const RowArgs<T>& a, int nb, int k, double* gout, hipStream_t stream) {
  hipLaunchKernelGGL(gauge_kernel<T>, dim3(nb), dim3(256), 0, stream, a, k, gout);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(const CombineDev* d, int npairs, long long maxn, T* out, hipStream_t stream) {
  dim3 grid((unsigned)((maxn + 255) / 256), npairs);
  hipLaunchKernelGGL(combine_kernel<T>, grid, dim3(256), 0, stream, d, out);
  return hipGetLastError();
}

template hipError_t launch_gauge<float>(const RowArgs<float>&, int, int, double*, hipStream_t);
template hipError_t launch_gauge<double>(const RowArgs<double>&, int, int, double*, hipStream_t);
template hipError_t launch_combine<float>(const CombineDev*, int, long long, float*, hipStream_t);
template hipError_t launch_combine<double>(const CombineDev*, int, long long, double*, hipStream_t);
template hipError_t launch_rows<float>(const RowArgs<float>&, int, hipStream_t);
template hipError_t launch_rows<double>(const RowArgs<double>&, int, hipStream_t);
template hipError_t launch_legendre<float>(const LegArgs<float>&, int, int, hipStream_t);
template hipError_t launch_legendre<double>(const LegArgs<double>&, int, int, hipStream_t);
template hipError_t launch_reduce<float>(const RowArgs<float>&, int, int, double*, double*, hipStream_t);
template hipError_t launch_reduce<double>(const RowArgs<double>&, int, int, double*, double*, hipStream_t);

}  // namespace shot
