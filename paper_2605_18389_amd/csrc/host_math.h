// Host-side float64 math for libshot plans: latitude quadrature, FFT
// factorisation and twiddles, heat multipliers, Legendre table and recurrence
// data.  Pure C++ (no HIP); everything here runs once per plan.
#pragma once

#include <cstdint>
#include <vector>

#if defined(__HIPCC__)
#define SHOT_HD __host__ __device__
#else
#define SHOT_HD
#endif

namespace shot {

// Row-split of one order's nr = L - m rows over the four waves of a Legendre
// workgroup: wave w handles rows [split_row(nr, w), split_row(nr, w + 1)),
// boundaries on multiples of 16 rows.  The blocks of 16 rows are dealt as
// evenly as they go (waves 0 .. nb16 % 4 - 1 take one more): the hardware puts
// the four waves of a workgroup on the four SIMDs of a compute unit starting
// at a SIMD it chooses, so with three workgroups per unit a split that leaves
// one light wave per workgroup always leaves some SIMD with only heavy waves.
inline SHOT_HD int split_row(int nr, int w) {
  const int nb16 = (nr + 15) / 16;
  const int base = nb16 / 4, rem = nb16 % 4;
  const int r = (w * base + (w < rem ? w : rem)) * 16;
  return r < nr ? r : nr;
}

// Rows of one parity of an order, padded to the 32-row K step of the
// matrix-core Legendre kernels.
inline SHOT_HD int mma_rpad(int n) { return (n + 31) / 32 * 32; }

// Gauss-Legendre nodes (descending, row 0 north) and weights (sum 2):
// the rows of a Gauss-Legendre grid sit at the roots of P_nlat (App. C.1).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Gauss-Lobatto rule (App. C.1, Lobatto): nodes at the poles and at the zeros
// of P'_{n-1} (descending, x = 1 first), weights 2 / (n (n-1) P_{n-1}(x_j)^2);
// exact to polynomial degree 2n - 3.  n >= 2.
void gauss_lobatto(int n, std::vector<double>& x, std::vector<double>& w);

// Clenshaw-Curtis rule on theta_j = j pi/(n-1), poles included (App. C.1).
void clenshaw_curtis(int n, std::vector<double>& x, std::vector<double>& w);

// Factors of any n >= 1: 4, 2, 3, 5 extracted first, then the remaining
// primes in increasing order (the device FFT runs those as generic stages).
std::vector<int> fft_factors(int n);

// In-place radix-2 FFT of a power-of-two length in double precision:
// a[k] <- sum_n a[n] exp(sign 2 pi i n k / n_len) (no scaling).
void fft_pow2(std::vector<double>& re, std::vector<double>& im, int sign);

// Bluestein tables for a transform of length n with convolution length m
// (a power of two >= 2n - 1): chirp[k] = exp(-i pi k^2 / n), k < n (angle
// reduced exactly as k^2 mod 2n), and bhat = FFT_m(b) / m with sign -1, where
// b[k] = b[m - k] = conj(chirp[k]) for k < n and 0 between; interleaved
// (re, im) pairs.
void bluestein_tables(int n, int m, std::vector<double>& chirp, std::vector<double>& bhat);

// HEALPix rings (Gorski et al. 2005), north to south, i = 1 .. 4 nside - 1:
// z = cos(colatitude) of the ring, its pixel count and the longitude of its
// first pixel in RING order.  North polar cap (i < nside): z = 1 - i^2/(3 nside^2),
// 4 i pixels from pi/(4 i); equatorial belt (nside <= i <= 2 nside): z = 4/3 -
// 2 i/(3 nside), 4 nside pixels from s pi/(4 nside), s = (i - nside + 1) mod 2;
// the southern rings mirror the northern ones (z -> -z).
void healpix_rings(int nside, std::vector<double>& z, std::vector<int>& npix, std::vector<double>& phi0);

// Offset of order m in the packed triangular (m, l) layout, l = m..L-1.
inline int64_t tri_offset(int64_t m, int64_t L) { return m * L - m * (m - 1) / 2; }

// Orthonormal associated Legendre values P̄_l^m(x_j) (App. B normalisation
// N_lm, no Condon-Shortley phase) for every m < L, l = m..L-1 and the given
// nodes, written row (tri_offset(m)+l-m) x column j into `tab` with row
// stride `ld`.  Computed per (m, x) by the normalised three-term recurrence in
// l, in float64, on `nthreads` host threads.
void legendre_rows(int L, const std::vector<double>& x, int ld, std::vector<double>& tab,
                   int nthreads);

// Data for generating P̄_l^m on the device with a two-operation recurrence.
// With P̄_l^m = alpha_l x P̄_{l-1}^m + beta_l P̄_{l-2}^m, define
// gamma_m = gamma_{m+1} = 1, gamma_l = beta_l gamma_{l-2}, R_l = P̄_l^m / gamma_l.
// Then R_l = (alpha_l gamma_{l-1}/gamma_l) x R_{l-1} + R_{l-2}.
// coef[tri(m,l)] = alpha_l gamma_{l-1}/gamma_l (l >= m+2; for l = m+1 it is the
// ratio P̄_{m+1}^m / (x P̄_m^m) = sqrt(2m+3)), gam[tri(m,l)] = gamma_l.
// seed[m*nx + j] = P̄_m^m(x_j) (may underflow to 0 where it is negligible).
void legendre_recurrence_data(int L, const std::vector<double>& x, std::vector<double>& coef,
                              std::vector<double>& gam, std::vector<double>& seed);

// One work item of the row-split Legendre kernel: rows [r_lo, r_hi) (row
// r = l - m) of order m, part s of the order's ns parts.  Parts of an order
// that has more than one sit at consecutive partial-buffer slots
// pslot - s .. pslot - s + ns - 1 (pslot = -1 when ns == 1).
struct SplitPartH {
  int m, r_lo, r_hi, s, ns, pslot;
};

// Work list for the row-split kernel: every order cut into parts of at most
// `part_rows` rows (a multiple of 64; <= 0: one part per order), sorted by
// decreasing length so that the longest work is dispatched first.  Returns the
// number of partial-buffer slots (parts of orders with ns > 1).
int split_schedule(int L, int part_rows, std::vector<SplitPartH>& parts);

// Dispatch order for the row-split kernel when every workgroup of a launch
// is resident at once: workgroup b lands on compute-unit slot b % ncu in
// round b / ncu, so the items dealt to one slot run side by side.  Returns
// order (a permutation of the item indices) such that the weights summed per
// slot are nearly equal: slots with fewer rounds take the heaviest items,
// each topped up toward the mean with the best-fitting remaining item; the
// others are filled heaviest first onto the least loaded slot; then swaps of
// single items between slots that do not raise the squared deviation from
// each slot's target even the loads out (deterministic: fixed-seed generator;
// slots with fewer rounds target short_factor of a full slot's load); within
// a slot the heaviest item runs in round 0.
std::vector<int> balanced_dispatch(const std::vector<int>& weight, int ncu, double short_factor = 0.95);

// Recurrence checkpoints for the row-split kernel: for every part k and wave
// w = 0..3 of its workgroup, the pair (R_{r0}, R_{r0-1}) of the rescaled
// recurrence at the wave's first row r0 = r_lo + split_row(r_hi - r_lo, w),
// stored at ck[((k*4 + w)*nx + j)*2 + {0,1}] ((0, 0) when the wave has no
// rows).  Evaluated with the same fused multiply-adds as the device recurrence.
void legendre_checkpoints(int L, const std::vector<double>& x, const std::vector<double>& coef,
                          const std::vector<double>& seed, const std::vector<SplitPartH>& parts,
                          std::vector<double>& ck, int nthreads);

}  // namespace shot
