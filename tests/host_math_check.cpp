// Host-logic checks for the row-split Legendre work lists (built with g++ by
// test_host_math.py against the library's host_math.cpp).  Prints "OK" and
// exits 0 when every check passes; prints the first failure otherwise.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "host_math.h"

using namespace shot;

static int fail(const char* what, long long a, long long b) {
  std::printf("FAIL %s (%lld, %lld)\n", what, a, b);
  return 1;
}

// Every row (m, r) of every order is covered by exactly one part; parts are
// sorted longest first; cut orders own consecutive partial slots.
static int check_schedule(int L, int part_rows) {
  std::vector<SplitPartH> parts;
  const int npb = split_schedule(L, part_rows, parts);
  std::vector<int> cover((size_t)L * L, 0);
  std::vector<int> slot_used(npb > 0 ? npb : 1, 0);
  for (size_t k = 0; k < parts.size(); ++k) {
    const SplitPartH& P = parts[k];
    if (k && parts[k - 1].r_hi - parts[k - 1].r_lo < P.r_hi - P.r_lo) return fail("order", (long long)k, 0);
    if (P.r_lo < 0 || P.r_hi > L - P.m || P.r_lo >= P.r_hi) return fail("range", P.m, P.r_lo);
    if (part_rows > 0 && P.r_hi - P.r_lo > part_rows) return fail("part length", P.m, P.r_hi - P.r_lo);
    if (P.r_lo % 16) return fail("part start alignment", P.m, P.r_lo);
    if (P.s < 0 || P.s >= P.ns) return fail("part index", P.m, P.s);
    if ((P.ns == 1) != (P.pslot < 0)) return fail("slot of whole order", P.m, P.pslot);
    if (P.ns > 1) {
      if (P.pslot >= npb) return fail("slot range", P.pslot, npb);
      ++slot_used[P.pslot];
    }
    for (int r = P.r_lo; r < P.r_hi; ++r) ++cover[(size_t)P.m * L + r];
  }
  for (int m = 0; m < L; ++m)
    for (int r = 0; r < L; ++r)
      if (cover[(size_t)m * L + r] != (r < L - m ? 1 : 0)) return fail("coverage", m, r);
  for (int q = 0; q < npb; ++q)
    if (slot_used[q] != 1) return fail("slot used once", q, slot_used[q]);
  // parts of one cut order: slots pslot - s consecutive
  for (const auto& P : parts)
    if (P.ns > 1)
      for (const auto& Q : parts)
        if (Q.m == P.m && Q.pslot - Q.s != P.pslot - P.s) return fail("slot base", P.m, Q.s);
  return 0;
}

// The dispatch order is a permutation whose per-slot weight sums (slot b % ncu)
// stay within `tol` of the mean, heaviest item first within a slot.
static int check_dispatch(int L, int ncu, double tol) {
  std::vector<int> w(L);
  for (int m = 0; m < L; ++m) w[m] = L - m;
  const std::vector<int> ord = balanced_dispatch(w, ncu);
  std::vector<int> seen(L, 0);
  for (int b = 0; b < L; ++b) {
    if (ord[b] < 0 || ord[b] >= L) return fail("dispatch range", b, ord[b]);
    ++seen[ord[b]];
  }
  for (int m = 0; m < L; ++m)
    if (seen[m] != 1) return fail("dispatch permutation", m, seen[m]);
  if (L <= ncu) return 0;
  std::vector<long long> load(ncu, 0);
  for (int b = 0; b < L; ++b) load[b % ncu] += w[ord[b]];
  long long mx = 0, tot = 0;
  for (long long v : load) { mx = std::max(mx, v); tot += v; }
  if ((double)mx > tol * (double)tot / ncu) return fail("dispatch balance", mx, tot / ncu);
  for (int b = ncu; b < L; ++b)
    if (w[ord[b]] > w[ord[b - ncu]]) return fail("heaviest first within a slot", b, ord[b]);
  return 0;
}

// Checkpoints: gamma_r * R_r reproduces the normalised table value P̄ (an
// independent recurrence) at each wave's first row r0 and the row before it,
// to 10 u L^1.5 of the row's largest value (the two recurrences round
// differently; near a zero of P̄ only an absolute comparison is meaningful).
static int check_checkpoints(int L, int nx, int part_rows) {
  std::vector<double> x, wq;
  gauss_legendre(nx, x, wq);
  std::vector<double> coef, gam, seed, tab, ck;
  legendre_recurrence_data(L, x, coef, gam, seed);
  const int ld = nx;
  legendre_rows(L, x, ld, tab, 2);
  std::vector<SplitPartH> parts;
  split_schedule(L, part_rows, parts);
  legendre_checkpoints(L, x, coef, seed, parts, ck, 2);
  const double tol = 10 * 1.1102230246251565e-16 * std::pow((double)L, 1.5);
  auto rowmax = [&](int64_t t) {
    double v = 0;
    for (int j = 0; j < nx; ++j) v = std::fmax(v, std::fabs(tab[(size_t)t * ld + j]));
    return v;
  };
  int checked = 0;
  for (size_t k = 0; k < parts.size(); ++k) {
    const SplitPartH& P = parts[k];
    const int len = P.r_hi - P.r_lo;
    for (int w = 0; w < 4; ++w) {
      const int r0 = P.r_lo + split_row(len, w);
      const int64_t t0 = tri_offset(P.m, L) + r0;
      const double s0 = r0 < P.r_hi ? rowmax(t0) : 0.0, s1 = (r0 < P.r_hi && r0 > 0) ? rowmax(t0 - 1) : 0.0;
      for (int j = 0; j < nx; ++j) {
        const double* c = ck.data() + ((k * 4 + w) * (size_t)nx + j) * 2;
        if (r0 >= P.r_hi) {
          if (c[0] != 0.0 || c[1] != 0.0) return fail("empty wave checkpoint", P.m, r0);
          continue;
        }
        if (std::fabs(gam[t0] * c[0] - tab[(size_t)t0 * ld + j]) > tol * s0)
          return fail("checkpoint R_r0", P.m * 10000 + r0, j);
        if (r0 > 0 && std::fabs(gam[t0 - 1] * c[1] - tab[(size_t)(t0 - 1) * ld + j]) > tol * s1)
          return fail("checkpoint R_r0-1", P.m * 10000 + r0, j);
        if (r0 == 0 && c[1] != 0.0) return fail("checkpoint below the seed", P.m, j);
        ++checked;
      }
    }
  }
  if (checked == 0) return fail("nothing checked", 0, 0);
  return 0;
}

// HEALPix rings: 12 nside^2 pixels on 4 nside - 1 rings, mirror symmetric,
// and equal-area: the cap above a ring's centres holds the rings above it and
// half of the ring, 2 pi (1 - z) = (pixels above + N/2) 4 pi / Npix.
static int check_healpix(int nside) {
  std::vector<double> z, phi0;
  std::vector<int> np;
  healpix_rings(nside, z, np, phi0);
  const int nr = 4 * nside - 1;
  if ((int)z.size() != nr) return fail("ring count", nside, (long long)z.size());
  long long tot = 0, above = 0;
  const double npix = 12.0 * nside * nside;
  for (int r = 0; r < nr; ++r) {
    tot += np[r];
    if (np[r] != np[nr - 1 - r] || std::fabs(z[r] + z[nr - 1 - r]) > 1e-15 ||
        std::fabs(phi0[r] - phi0[nr - 1 - r]) > 1e-15)
      return fail("mirror symmetry", nside, r);
    if (phi0[r] < 0 || phi0[r] >= 2 * M_PI / np[r]) return fail("first longitude", nside, r);
    const double cap = 2 * M_PI * (1 - z[r]), want = (above + np[r] / 2.0) * 4 * M_PI / npix;
    if (std::fabs(cap - want) > 1e-13) return fail("equal area", nside, r);
    above += np[r];
  }
  if (tot != 12LL * nside * nside) return fail("pixel count", nside, tot);
  return 0;
}

// Factor lists multiply back to n, 4/2/3/5 first, then primes ascending.
static int check_factors() {
  for (int n = 1; n <= 4096; ++n) {
    const std::vector<int> f = fft_factors(n);
    long long prod = 1;
    int stage = 0;  // 0: 4/2/3/5 section, 1: other primes
    int last = 0;
    for (int r : f) {
      prod *= r;
      const bool small = (r == 2 || r == 3 || r == 4 || r == 5);
      if (!small) {
        if (r < 7) return fail("factor", n, r);
        for (int d = 2; d * d <= r; ++d)
          if (r % d == 0) return fail("composite factor", n, r);
        if (stage == 1 && r < last) return fail("factor order", n, r);
        stage = 1;
        last = r;
      } else if (stage == 1) {
        return fail("small factor after a prime", n, r);
      }
    }
    if (prod != n) return fail("factor product", n, prod);
  }
  return 0;
}

// Gauss-Lobatto: the 5-point textbook rule, and exactness to degree 2n - 3.
static int check_lobatto() {
  std::vector<double> x, w;
  gauss_lobatto(5, x, w);
  const double xs[5] = {1.0, std::sqrt(3.0 / 7.0), 0.0, -std::sqrt(3.0 / 7.0), -1.0};
  const double ws[5] = {0.1, 49.0 / 90.0, 32.0 / 45.0, 49.0 / 90.0, 0.1};
  for (int j = 0; j < 5; ++j)
    if (std::fabs(x[j] - xs[j]) > 1e-15 || std::fabs(w[j] - ws[j]) > 1e-14) return fail("lobatto 5-point", j, 0);
  for (int n : {3, 8, 33, 181}) {
    gauss_lobatto(n, x, w);
    for (int k = 0; k <= 2 * n - 3; k += 2) {
      double s = 0;
      for (int j = 0; j < n; ++j) s += w[j] * std::pow(x[j], k);
      if (std::fabs(s - 2.0 / (k + 1)) > 1e-12) return fail("lobatto exactness", n, k);
    }
  }
  return 0;
}

// Bluestein tables: the length-n DFT assembled from them (pre-multiply by the
// chirp, power-of-two FFT, multiply by the filter spectrum, inverse FFT,
// post-multiply; conjugated tables for the inverse direction) equals the
// direct sum to 1e-12 of its largest value, in both directions.
static int check_bluestein(int n) {
  int m = 1;
  while (m < 2 * n - 1) m *= 2;
  std::vector<double> ch, bh;
  bluestein_tables(n, m, ch, bh);
  std::vector<double> xr(n), xi(n);
  for (int j = 0; j < n; ++j) {
    xr[j] = std::sin(0.37 * j * j + 1.0);
    xi[j] = std::cos(1.3 * j + 0.2);
  }
  for (int sign : {-1, 1}) {
    const double cs = sign < 0 ? 1.0 : -1.0;  // conjugate the tables for sign +1
    std::vector<double> ar(m, 0.0), ai(m, 0.0);
    for (int j = 0; j < n; ++j) {
      const double cr = ch[2 * j], ci = cs * ch[2 * j + 1];
      ar[j] = xr[j] * cr - xi[j] * ci;
      ai[j] = xr[j] * ci + xi[j] * cr;
    }
    fft_pow2(ar, ai, -1);
    for (int k = 0; k < m; ++k) {
      const double fr = bh[2 * k], fi = cs * bh[2 * k + 1];
      const double r = ar[k] * fr - ai[k] * fi, i = ar[k] * fi + ai[k] * fr;
      ar[k] = r;
      ai[k] = i;
    }
    fft_pow2(ar, ai, 1);
    double err = 0, big = 0;
    for (int k = 0; k < n; ++k) {
      const double cr = ch[2 * k], ci = cs * ch[2 * k + 1];
      const double yr = ar[k] * cr - ai[k] * ci, yi = ar[k] * ci + ai[k] * cr;
      long double dr = 0, di = 0;
      for (int j = 0; j < n; ++j) {
        const long double ang = (long double)sign * 2.0L * (long double)M_PI * (long double)(((long long)j * k) % n) / n;
        dr += xr[j] * cosl(ang) - xi[j] * sinl(ang);
        di += xr[j] * sinl(ang) + xi[j] * cosl(ang);
      }
      err = std::fmax(err, std::hypot(yr - (double)dr, yi - (double)di));
      big = std::fmax(big, std::hypot((double)dr, (double)di));
    }
    if (err > 1e-12 * big) return fail("bluestein", n, sign);
  }
  return 0;
}

int main() {
  int rc = 0;
  for (int L : {1, 15, 16, 17, 90, 181, 720})
    for (int pr : {0, 64, 128, 384}) rc |= check_schedule(L, pr);
  rc |= check_dispatch(720, 256, 1.015);  // full slots target 1.0095 x the mean (two-item slots 0.95 of that)
  rc |= check_dispatch(360, 256, 1.45);  // one order of 360 rows exceeds the mean (254)
  rc |= check_dispatch(100, 256, 1e9);
  rc |= check_checkpoints(80, 40, 0);
  rc |= check_checkpoints(80, 40, 64);
  rc |= check_checkpoints(150, 75, 64);
  for (int nside : {1, 2, 3, 7, 8, 64, 256}) rc |= check_healpix(nside);
  rc |= check_factors();
  for (int n : {268, 404, 1004}) rc |= check_bluestein(n);
  rc |= check_lobatto();
  if (!rc) std::printf("OK\n");
  return rc;
}
