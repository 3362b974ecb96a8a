// Host-side float64 math for libshot plans (see host_math.h).
#include "host_math.h"

#include <algorithm>
#include <numeric>
#include <queue>
#include <random>
#include <cmath>
#include <thread>

namespace shot {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  // Newton's method on P_n, P_n evaluated by Bonnet's recurrence; the start
  // values cos(pi (i + 3/4)/(n + 1/2)) are already ordered north to south.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pn = 0, dpn = 1;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      pn = (n == 0) ? 1.0 : p1;
      dpn = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = pn / dpn;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < n; ++k) {
      double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    dpn = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
  // enforce the exact equatorial symmetry the folded kernels rely on
  for (int i = 0; i < n / 2; ++i) {
    double xs = 0.5 * (x[i] - x[n - 1 - i]);
    double ws = 0.5 * (w[i] + w[n - 1 - i]);
    x[i] = xs;
    x[n - 1 - i] = -xs;
    w[i] = w[n - 1 - i] = ws;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

void clenshaw_curtis(int n, std::vector<double>& x, std::vector<double>& w) {
  // w_j = c_j/N (1 - sum_{k=1}^{N/2} b_k cos(2 k theta_j)/(4k^2 - 1)), N = n-1,
  // c_j = 1 at the poles and 2 elsewhere, b_k = 1 for k = N/2 and 2 otherwise.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const int N = n - 1;
  for (int j = 0; j < n; ++j) {
    const double th = M_PI * j / N;
    double s = 0.0;
    for (int k = 1; 2 * k <= N; ++k) {
      const double b = (2 * k == N) ? 1.0 : 2.0;
      s += b * std::cos(2.0 * k * th) / (4.0 * k * k - 1.0);
    }
    w[j] = ((j == 0 || j == N) ? 1.0 : 2.0) / N * (1.0 - s);
    x[j] = std::cos(th);
  }
  for (int i = 0; i < n / 2; ++i) {
    double xs = 0.5 * (x[i] - x[n - 1 - i]);
    double ws = 0.5 * (w[i] + w[n - 1 - i]);
    x[i] = xs;
    x[n - 1 - i] = -xs;
    w[i] = w[n - 1 - i] = ws;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

void gauss_lobatto(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const int N = n - 1;
  // P_N and P_N' by the three-term recurrence (plain Legendre polynomials)
  auto pn = [N](double t, double& p, double& dp) {
    double p0 = 1.0, p1 = t;
    if (N == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 1; k < N; ++k) {
      const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    p = p1;
    dp = N * (t * p1 - p0) / (t * t - 1.0);
  };
  x[0] = 1.0;
  x[N] = -1.0;
  for (int j = 1; j < N; ++j) {
    // Newton on P_N' from the Chebyshev-Lobatto point; Legendre's equation gives
    // (1 - t^2) P_N'' = 2 t P_N' - N (N + 1) P_N
    double t = std::cos(M_PI * j / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      pn(t, p, dp);
      const double d2p = (2.0 * t * dp - N * (N + 1.0) * p) / (1.0 - t * t);
      const double dt = dp / d2p;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[j] = t;
  }
  for (int j = 0; j < n; ++j) {
    double p;
    if (j == 0) p = 1.0;
    else if (j == N) p = (N % 2) ? -1.0 : 1.0;
    else {
      double dp;
      pn(x[j], p, dp);
    }
    w[j] = 2.0 / (n * (double)N * p * p);
  }
}

std::vector<int> fft_factors(int n) {
  std::vector<int> f;
  if (n < 1) return f;
  for (int r : {4, 2, 3, 5})
    while (n % r == 0) {
      f.push_back(r);
      n /= r;
    }
  for (int p = 7; n > 1; p += 2)
    while (n % p == 0) {
      f.push_back(p);
      n /= p;
    }
  return f;
}

void fft_pow2(std::vector<double>& re, std::vector<double>& im, int sign) {
  const size_t n = re.size();
  for (size_t i = 1, j = 0; i < n; ++i) {  // bit reversal
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      std::swap(re[i], re[j]);
      std::swap(im[i], im[j]);
    }
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t k = 0; k < len / 2; ++k) {
      const long double ang = (long double)sign * 2.0L * (long double)M_PI * (long double)k / (long double)len;
      const double wr = (double)cosl(ang), wi = (double)sinl(ang);
      for (size_t i = 0; i < n; i += len) {
        const size_t u = i + k, v = i + k + len / 2;
        const double xr = re[v] * wr - im[v] * wi, xi = re[v] * wi + im[v] * wr;
        re[v] = re[u] - xr;
        im[v] = im[u] - xi;
        re[u] += xr;
        im[u] += xi;
      }
    }
  }
}

void bluestein_tables(int n, int m, std::vector<double>& chirp, std::vector<double>& bhat) {
  chirp.assign(2 * (size_t)n, 0.0);
  std::vector<double> br(m, 0.0), bi(m, 0.0);
  for (int k = 0; k < n; ++k) {
    const long long q = ((long long)k * k) % (2LL * n);
    const long double ang = -(long double)M_PI * (long double)q / (long double)n;
    chirp[2 * k] = (double)cosl(ang);
    chirp[2 * k + 1] = (double)sinl(ang);
    br[k] = chirp[2 * k];
    bi[k] = -chirp[2 * k + 1];
    if (k > 0) {
      br[m - k] = br[k];
      bi[m - k] = bi[k];
    }
  }
  fft_pow2(br, bi, -1);
  bhat.assign(2 * (size_t)m, 0.0);
  for (int k = 0; k < m; ++k) {
    bhat[2 * k] = br[k] / m;
    bhat[2 * k + 1] = bi[k] / m;
  }
}

void healpix_rings(int nside, std::vector<double>& z, std::vector<int>& npix, std::vector<double>& phi0) {
  const int nr = 4 * nside - 1;
  z.assign(nr, 0.0);
  npix.assign(nr, 0);
  phi0.assign(nr, 0.0);
  const double ns = (double)nside;
  for (int r = 0; r < nr; ++r) {
    const int i = r + 1;
    const int k = i <= 2 * nside ? i : 4 * nside - i;  // the northern ring of the mirror pair
    double zk;
    if (k < nside) {
      zk = 1.0 - (double)k * k / (3.0 * ns * ns);
      npix[r] = 4 * k;
      phi0[r] = M_PI / (4.0 * k);
    } else {
      zk = 4.0 / 3.0 - 2.0 * k / (3.0 * ns);
      npix[r] = 4 * nside;
      phi0[r] = ((k - nside + 1) % 2) * M_PI / (4.0 * ns);
    }
    z[r] = i <= 2 * nside ? zk : -zk;
  }
}

namespace {

// One order m: P̄_l^m(x) for l = m..L-1 at a single node, into out[l-m].
void legendre_column(int L, int m, double x, double* out, int64_t stride) {
  const double s = std::sqrt(std::max(0.0, 1.0 - x * x));
  double pmm = 1.0 / std::sqrt(4.0 * M_PI);
  for (int k = 1; k <= m; ++k) pmm *= std::sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
  out[0] = pmm;
  if (L - m < 2) return;
  double p1 = std::sqrt(2.0 * m + 3.0) * x * pmm;
  out[stride] = p1;
  double p2 = pmm;
  for (int l = m + 2; l < L; ++l) {
    const double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
    const double b = std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
    const double p = a * (x * p1 - b * p2);
    out[(int64_t)(l - m) * stride] = p;
    p2 = p1;
    p1 = p;
  }
}

}  // namespace

void legendre_rows(int L, const std::vector<double>& x, int ld, std::vector<double>& tab,
                   int nthreads) {
  const int nx = (int)x.size();
  const int64_t rows = (int64_t)L * (L + 1) / 2;
  tab.assign(rows * ld, 0.0);
  nthreads = std::max(1, nthreads);
  std::vector<std::thread> pool;
  for (int tid = 0; tid < nthreads; ++tid) {
    pool.emplace_back([&, tid]() {
      for (int m = tid; m < L; m += nthreads) {
        double* base = tab.data() + tri_offset(m, L) * ld;
        for (int j = 0; j < nx; ++j) legendre_column(L, m, x[j], base + j, ld);
      }
    });
  }
  for (auto& t : pool) t.join();
}

void legendre_recurrence_data(int L, const std::vector<double>& x, std::vector<double>& coef,
                              std::vector<double>& gam, std::vector<double>& seed) {
  const int nx = (int)x.size();
  const int64_t rows = (int64_t)L * (L + 1) / 2;
  coef.assign(rows, 0.0);
  gam.assign(rows, 1.0);
  seed.assign((int64_t)L * nx, 0.0);
  for (int m = 0; m < L; ++m) {
    const int64_t o = tri_offset(m, L);
    // gamma and the x-coefficient of the rescaled recurrence
    for (int l = m; l < L; ++l) {
      if (l == m) {
        gam[o] = 1.0;
        coef[o] = 0.0;
      } else if (l == m + 1) {
        gam[o + 1] = 1.0;
        coef[o + 1] = std::sqrt(2.0 * m + 3.0);
      } else {
        const double alpha = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double beta = -std::sqrt((2.0 * l + 1.0) * ((l - 1.0) * (l - 1.0) - (double)m * m) /
                                       ((2.0 * l - 3.0) * ((double)l * l - (double)m * m)));
        gam[o + (l - m)] = beta * gam[o + (l - m) - 2];
        coef[o + (l - m)] = alpha * gam[o + (l - m) - 1] / gam[o + (l - m)];
      }
    }
    for (int j = 0; j < nx; ++j) {
      const double s = std::sqrt(std::max(0.0, 1.0 - x[j] * x[j]));
      double pmm = 1.0 / std::sqrt(4.0 * M_PI);
      for (int k = 1; k <= m; ++k) pmm *= std::sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
      seed[(int64_t)m * nx + j] = pmm;
    }
  }
}

}  // namespace shot

namespace shot {

int split_schedule(int L, int part_rows, std::vector<SplitPartH>& parts) {
  parts.clear();
  int nslot = 0;
  for (int m = 0; m < L; ++m) {
    const int nr = L - m;
    const int pr = part_rows > 0 ? part_rows : nr;
    const int ns = (nr + pr - 1) / pr;
    for (int s = 0; s < ns; ++s) {
      const int lo = s * pr, hi = std::min(nr, lo + pr);
      parts.push_back({m, lo, hi, s, ns, ns > 1 ? nslot + s : -1});
    }
    if (ns > 1) nslot += ns;
  }
  std::stable_sort(parts.begin(), parts.end(), [](const SplitPartH& a, const SplitPartH& b) {
    return a.r_hi - a.r_lo > b.r_hi - b.r_lo;
  });
  return nslot;
}

std::vector<int> balanced_dispatch(const std::vector<int>& weight, int ncu, double short_factor) {
  const int n = (int)weight.size();
  std::vector<int> order(n);
  for (int b = 0; b < n; ++b) order[b] = b;
  if (n <= ncu) return order;
  // items by decreasing weight
  std::vector<int> items(n);
  std::iota(items.begin(), items.end(), 0);
  std::stable_sort(items.begin(), items.end(), [&](int a, int b) { return weight[a] > weight[b]; });
  const int rounds = (n + ncu - 1) / ncu;
  std::vector<int> cap(ncu, 0);
  for (int s = 0; s < ncu; ++s)
    for (int r = 0; r < rounds; ++r)
      if (r * ncu + s < n) ++cap[s];
  double total = 0;
  for (int w : weight) total += w;
  const double target = total / ncu;
  std::vector<std::vector<int>> slot(ncu);
  std::vector<long long> load(ncu, 0);
  std::vector<char> used(n, 0);
  size_t next = 0;
  const int cmin = *std::min_element(cap.begin(), cap.end());
  const int cmax = *std::max_element(cap.begin(), cap.end());
  if (cmin < cmax) {
    for (int s = 0; s < ncu; ++s) {
      if (cap[s] != cmin) continue;
      while (used[items[next]]) ++next;
      const int a = items[next];
      used[a] = 1;
      slot[s].push_back(a);
      load[s] += weight[a];
      for (int k = 1; k < cmin; ++k) {
        const double need = target - (double)load[s];
        int best = -1;
        for (int i = 0; i < n; ++i)
          if (!used[i] && (best < 0 || std::fabs(weight[i] - need) < std::fabs(weight[best] - need))) best = i;
        used[best] = 1;
        slot[s].push_back(best);
        load[s] += weight[best];
      }
    }
  }
  using E = std::pair<long long, int>;
  std::priority_queue<E, std::vector<E>, std::greater<E>> pq;
  for (int s = 0; s < ncu; ++s)
    if ((int)slot[s].size() < cap[s]) pq.push({load[s], s});
  for (int i : items) {
    if (used[i]) continue;
    const E e = pq.top();
    pq.pop();
    const int s = e.second;
    slot[s].push_back(i);
    load[s] += weight[i];
    used[i] = 1;
    if ((int)slot[s].size() < cap[s]) pq.push({load[s], s});
  }
  // The filling above leaves a staircase of slot loads (at L = 720: 930 to
  // 1089 rows against a mean of 1014) that no swap lowering the heaviest slot
  // alone can flatten.  Random swaps of one item between two slots (slot sizes
  // kept) that do not raise the sum of squared deviations from the slots'
  // targets accept the sideways moves that can (max 1017 at L = 720); the
  // generator's fixed seed keeps the plan deterministic.  A slot with fewer
  // rounds runs fewer waves per SIMD, which hide each other's latency less:
  // its target is short_factor of a full slot's (the recurrence kernel at
  // L = 720: 0.95 gives 34.85 -> 34.52 us per launch, 0.9 is slower again).
  std::vector<double> tgt(ncu);
  {
    double wsum = 0.0;
    for (int s = 0; s < ncu; ++s) wsum += cap[s] == cmax ? 1.0 : short_factor;
    for (int s = 0; s < ncu; ++s) tgt[s] = total / wsum * (cap[s] == cmax ? 1.0 : short_factor);
  }
  std::mt19937 rng(20240607u);
  auto sq = [](double v) { return v * v; };
  for (int sweep = 0; sweep < 200; ++sweep) {  // a few ms at L = 720
    for (int k = 0; k < 8 * ncu; ++k) {
      const int s = (int)(rng() % (unsigned)ncu), t = (int)(rng() % (unsigned)ncu);
      if (s == t || slot[s].empty() || slot[t].empty()) continue;
      const int i = (int)(rng() % slot[s].size()), j = (int)(rng() % slot[t].size());
      const long long d = (long long)weight[slot[s][i]] - weight[slot[t][j]];
      if (d == 0) continue;
      const double before = sq((double)load[s] - tgt[s]) + sq((double)load[t] - tgt[t]);
      const double after = sq((double)(load[s] - d) - tgt[s]) + sq((double)(load[t] + d) - tgt[t]);
      if (after <= before) {
        std::swap(slot[s][i], slot[t][j]);
        load[s] -= d;
        load[t] += d;
      }
    }
  }
  for (int s = 0; s < ncu; ++s) {
    std::stable_sort(slot[s].begin(), slot[s].end(), [&](int a, int b) { return weight[a] > weight[b]; });
    for (int r = 0; r < (int)slot[s].size(); ++r) order[r * ncu + s] = slot[s][r];
  }
  return order;
}

void legendre_checkpoints(int L, const std::vector<double>& x, const std::vector<double>& coef,
                          const std::vector<double>& seed, const std::vector<SplitPartH>& parts,
                          std::vector<double>& ck, int nthreads) {
  const int nx = (int)x.size();
  const size_t np = parts.size();
  ck.assign(np * 4 * nx * 2, 0.0);
  // wave starts grouped by order, in increasing row
  std::vector<std::vector<std::pair<int, size_t>>> by_m(L);
  for (size_t k = 0; k < np; ++k) {
    const SplitPartH& P = parts[k];
    const int len = P.r_hi - P.r_lo;
    for (int w = 0; w < 4; ++w) {
      const int r0 = P.r_lo + split_row(len, w);
      if (r0 < P.r_hi) by_m[P.m].push_back({r0, k * 4 + w});
    }
  }
  for (auto& v : by_m) std::sort(v.begin(), v.end());
  nthreads = std::max(1, nthreads);
  std::vector<std::thread> pool;
  for (int tid = 0; tid < nthreads; ++tid) {
    pool.emplace_back([&, tid]() {
      for (int m = tid; m < L; m += nthreads) {
        const double* c = coef.data() + tri_offset(m, L);
        for (int j = 0; j < nx; ++j) {
          double r1 = seed[(size_t)m * nx + j], r2 = 0.0;
          int r = 0;
          for (const auto& st : by_m[m]) {
            while (r < st.first) {
              ++r;
              const double rn = std::fma(c[r] * x[j], r1, r2);
              r2 = r1;
              r1 = rn;
            }
            double* dst = ck.data() + (st.second * nx + j) * 2;
            dst[0] = r1;
            dst[1] = r2;
          }
        }
      }
    });
  }
  for (auto& t : pool) t.join();
}

}  // namespace shot

namespace shot {

void legendre_checkpoints(int L, const std::vector<double>& x, const std::vector<double>& coef,
                          const std::vector<double>& seed, std::vector<double>& ck, int nthreads) {
  const int nx = (int)x.size();
  ck.assign((size_t)L * 4 * nx * 2, 0.0);
  nthreads = std::max(1, nthreads);
  std::vector<std::thread> pool;
  for (int tid = 0; tid < nthreads; ++tid) {
    pool.emplace_back([&, tid]() {
      for (int m = tid; m < L; m += nthreads) {
        const int nr = L - m;
        const double* c = coef.data() + tri_offset(m, L);
        for (int j = 0; j < nx; ++j) {
          double r1 = seed[(size_t)m * nx + j], r2 = 0.0;
          int r = 0;
          for (int w = 0; w < 4; ++w) {
            const int r0 = split_row(nr, w);
            if (r0 >= nr) break;
            while (r < r0) {
              ++r;
              const double rn = std::fma(c[r] * x[j], r1, r2);
              r2 = r1;
              r1 = rn;
            }
            double* dst = ck.data() + (((size_t)m * 4 + w) * nx + j) * 2;
            dst[0] = r1;
            dst[1] = r2;
          }
        }
      }
    });
  }
  for (auto& t : pool) t.join();
}

}  // namespace shot
