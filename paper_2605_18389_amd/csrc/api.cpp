// C ABI of libshot (declared in include/shot.h): plans, heat apply, Sinkhorn
// solves (Alg. 1), divergence (Def. 2.3) and its gradient (Sec. 4.2.2).
//
// Host-side orchestration only: every arithmetic step of the hot path runs in
// the HIP kernels of kernels.hip; the host computes plan-time float64 data
// (quadrature, Legendre tables or recurrence data, heat multipliers) and the
// final float64 combination of three scalar costs into a divergence.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <mutex>
#include <thread>
#include <map>
#include <vector>

#include "../../include/shot.h"
#include "host_math.h"
#include "shot_internal.h"

using namespace shot;

// Hash of the sources the library was built from (set by the build script).
#ifndef SHOT_SOURCE_HASH
#define SHOT_SOURCE_HASH "unknown"
#endif

namespace {

// Work list of the row-split Legendre kernel (parts, their checkpoints).
struct SplitSched {
  SplitPartH* d_parts = nullptr;
  double* d_ck = nullptr;
  int n = 0, maxlen = 0, npb = 0;
};

struct GridRec {
  shot_grid_desc d{};
  int h = 0, hpad = 0;
  std::vector<double> x, w;
  std::vector<double> aw_host;  // area weight of each row pair, double precision
  std::vector<int> fac;
  int tab_kind = TAB_F32;
  void* d_tab = nullptr;
  int* d_morder = nullptr;           // [L] order run by MFMA workgroup column b (rows balanced over units)
  double* d_xs = nullptr;
  double* d_rcoef = nullptr;
  double* d_rgam = nullptr;
  double* d_rseed = nullptr;
  SplitSched sw;                     // one part per order
  SplitSched ss;                     // long orders cut into parts (small batches)
  int2* d_cut = nullptr;             // [L] (parts, first partial slot) of the cut work list
  void* d_pbuf = nullptr;            // partial sums of cut orders, 4 chunks of 2 items
  void* d_aw = nullptr;
  void* d_tw = nullptr;
  // HEALPix: ring pairs, twiddles of every ring length, e^{i m phi0} per (pair, m)
  bool hp = false;
  int nside = 0;
  std::vector<int> ring_npix;
  std::vector<double> ring_phi0;
  RingDev* d_ring = nullptr;
  int* d_rpair = nullptr;            // ring pair run by row workgroup column b (cost-balanced over XCDs)
  void* d_ring_tw = nullptr;
  void* d_ring_ph = nullptr;
  void* d_ring_blu = nullptr;        // Bluestein chirps and filter spectra of long-prime rings
  int ring_nbuf = 0;                 // LDS length of a ring FFT buffer
  int tune_ib = 0;   // Legendre items per workgroup (0 = automatic)
  int tune_jpt = 0;  // recurrence chains per thread (0 = automatic); table grids: MFMA column
                     // tiles (1, 2, 4), 0 = automatic, -1 = VALU kernel only
  int64_t n() const { return hp ? 12LL * nside * nside : (int64_t)d.nlat * d.nlon; }
};

// float32 or bfloat16 table plans run the matrix-core table kernel
static bool mma_table(const GridRec& g) {
  return g.d_tab != nullptr && (g.tab_kind == TAB_F32 || g.tab_kind == TAB_BF16);
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Timed {
  hipEvent_t a, b;
  int cls;
};

}  // namespace

struct shot_plan_s {
  int prec = SHOT_FP32;
  int dev = 0;
  std::vector<GridRec> grids;
  DevBuf ws;  // call workspace arena (grown on demand)
  DevBuf ws2; // gradient workspace arena (adjoint history, checkpoints, accumulators)
  bool prof = false;
  std::vector<Timed> timed;
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  int leg_ib = 0;  // 0 = choose automatically
  // fixed-T solve loops are captured once into a HIP graph and replayed
  bool graphs = true;
  hipStream_t cap = nullptr;
  // side streams of a captured solve: one branch per grid group after the
  // first, forked from and joined back into the capture stream
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> bev;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<long long> gkey;
};

namespace {
void drop_graph(shot_plan_s* P) {
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->gexec = nullptr;
  P->graph = nullptr;
  P->gkey.clear();
}
}  // namespace

namespace {

thread_local char g_last_error[512] = "";

shot_status hip_fail(hipError_t e, const char* what, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s (line %d): %s (%d)", what, line,
           hipGetErrorString(e), (int)e);
  return SHOT_E_HIP;
}

#define HIP_TRY(expr)                                         \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__); \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

shot_status grow(DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return SHOT_OK;
  if (b.p) {
    if (hipFree(b.p) != hipSuccess) return SHOT_E_HIP;
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    hip_fail(e, "hipMalloc(workspace)", __LINE__);
    return SHOT_E_NOMEM;
  }
  b.bytes = bytes;
  return SHOT_OK;
}

template <typename T>
size_t real_size() { return sizeof(T); }

size_t field_elem(const shot_plan_s* P) { return P->prec == SHOT_FP64 ? 8 : 4; }

hipEvent_t take_event(shot_plan_s* P) {
  if (P->evnext == P->evpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    P->evpool.push_back(e);
  }
  return P->evpool[P->evnext++];
}

// Time one launch with dispatch-attached events when profiling is on.
struct ProfScope {
  shot_plan_s* P;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(shot_plan_s* P_, hipStream_t, int cls_) : P(P_), cls(cls_) {
    if (P->prof) {
      a = take_event(P);
      b = take_event(P);
      if (a && b) {
        set_launch_events(a, b);
        P->timed.push_back({a, b, cls});
      }
    }
  }
};

// Upload host vector -> new device allocation.
template <typename V>
shot_status upload(void** dst, const std::vector<V>& src, hipStream_t s) {
  *dst = nullptr;
  if (src.empty()) return SHOT_OK;
  hipError_t e = hipMalloc(dst, src.size() * sizeof(V));
  if (e != hipSuccess) { *dst = nullptr; hip_fail(e, "hipMalloc", __LINE__); return SHOT_E_NOMEM; }
  HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return SHOT_OK;
}

uint16_t to_bf16(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest even
  return (uint16_t)(u >> 16);
}

void free_grid(GridRec& g) {
  for (void* p : {g.d_tab, (void*)g.d_xs, (void*)g.d_rcoef, (void*)g.d_rgam,
                  (void*)g.d_rseed, (void*)g.sw.d_parts, (void*)g.sw.d_ck, (void*)g.ss.d_parts,
                  (void*)g.ss.d_ck, (void*)g.d_morder, (void*)g.d_ring, (void*)g.d_rpair, g.d_ring_tw, g.d_ring_ph, g.d_ring_blu, (void*)g.d_cut, g.d_pbuf, g.d_aw, g.d_tw})
    if (p) (void)hipFree(p);
  g.d_tab = g.d_aw = g.d_tw = g.d_pbuf = g.d_ring_tw = g.d_ring_ph = g.d_ring_blu = nullptr;
  g.d_morder = nullptr;
  g.d_ring = nullptr;
  g.d_rpair = nullptr;
  g.d_xs = g.d_rcoef = g.d_rgam = g.d_rseed = nullptr;
  g.sw = SplitSched{};
  g.ss = SplitSched{};
  g.d_cut = nullptr;
}

shot_status build_grid(shot_plan_s* P, GridRec& g, int leg_mode, hipStream_t s) {
  const auto& d = g.d;
  g.hp = d.kind == SHOT_GRID_HEALPIX;
  if (g.hp) {
    // rings (z, pixel count, first longitude); w_j = the ring's area / (2 pi)
    g.nside = d.nlon / 4;
    healpix_rings(g.nside, g.x, g.ring_npix, g.ring_phi0);
    g.w.resize(d.nlat);
    const double npix = 12.0 * g.nside * g.nside;
    for (int r = 0; r < d.nlat; ++r) g.w[r] = 2.0 * g.ring_npix[r] / npix;
  } else if (d.kind == SHOT_GRID_GAUSS_LEGENDRE) {
    gauss_legendre(d.nlat, g.x, g.w);
  } else if (d.kind == SHOT_GRID_LOBATTO) {
    gauss_lobatto(d.nlat, g.x, g.w);
  } else {
    clenshaw_curtis(d.nlat, g.x, g.w);
  }
  g.h = (d.nlat + 1) / 2;
  // table rows padded to the matrix-core K step (32) for fp32/bf16 tables
  g.hpad = P->prec == SHOT_FP64 ? (g.h + 3) / 4 * 4 : (g.h + 31) / 32 * 32;
  g.fac = g.hp ? std::vector<int>() : fft_factors(d.nlon);
  const bool f64 = P->prec == SHOT_FP64;
  // area weights of rows 0..h-1 and twiddles in field precision
  std::vector<double> aw(g.h);
  for (int j = 0; j < g.h; ++j)
    aw[j] = g.hp ? 4.0 * M_PI / (12.0 * g.nside * g.nside) : g.w[j] * 2.0 * M_PI / d.nlon;
  g.aw_host = aw;
  if (g.hp) {
    // ring pairs: geometry, twiddles per distinct length (4k pixels, k = 1..nside), phases
    std::vector<RingDev> rings(g.h);
    std::vector<long long> twoff(g.nside + 1, -1);
    std::vector<double> rtw, blu;
    std::map<int, long long> mtwoff, bluoff;
    int nbuf = d.nlon;
    std::vector<long long> start(d.nlat + 1, 0);
    for (int r = 0; r < d.nlat; ++r) start[r + 1] = start[r] + g.ring_npix[r];
    for (int j = 0; j < g.h; ++j) {
      RingDev& R = rings[j];
      const int len = g.ring_npix[j];
      R.len = len;
      R.off1 = (int)start[j];
      R.off2 = (int)start[d.nlat - 1 - j];
      const int k = len / 4;
      if (twoff[k] < 0) {
        twoff[k] = (long long)rtw.size() / 2;
        for (int q = 0; q < len; ++q) {
          const long double ang = -2.0L * (long double)M_PI * (long double)q / (long double)len;
          rtw.push_back((double)cosl(ang));
          rtw.push_back((double)sinl(ang));
        }
      }
      R.twoff = (int)twoff[k];
      const std::vector<int> f = fft_factors(len);
      if ((int)f.size() > RING_MAXFAC) return SHOT_E_UNSUPPORTED;
      R.nfac = (int)f.size();
      for (int q = 0; q < RING_MAXFAC; ++q) R.fac[q] = q < R.nfac ? f[q] : 0;
      // a prime factor above 64 (polar rings of 4p pixels beyond Nside 64):
      // Bluestein, a cyclic convolution of power-of-two length M >= 2 len - 1
      R.bm = 0;
      if (f.back() > 64) {
        int M = 1;
        while (M < 2 * len - 1) M *= 2;
        R.bm = M;
        const std::vector<int> fm = fft_factors(M);
        R.bm_nfac = (int)fm.size();
        for (int q = 0; q < RING_MAXFAC; ++q) R.bm_fac[q] = q < R.bm_nfac ? fm[q] : 0;
        if (!mtwoff.count(M)) {
          mtwoff[M] = (long long)rtw.size() / 2;
          for (int q = 0; q < M; ++q) {
            const long double ang = -2.0L * (long double)M_PI * (long double)q / (long double)M;
            rtw.push_back((double)cosl(ang));
            rtw.push_back((double)sinl(ang));
          }
        }
        R.bm_twoff = (int)mtwoff[M];
        if (!bluoff.count(len)) {
          std::vector<double> ch, bh;
          bluestein_tables(len, M, ch, bh);
          bluoff[len] = (long long)blu.size() / 2;
          blu.insert(blu.end(), ch.begin(), ch.end());
          blu.insert(blu.end(), bh.begin(), bh.end());
        }
        R.ch_off = (int)bluoff[len];
        R.bh_off = R.ch_off + len;
        nbuf = std::max(nbuf, M);
      }
    }
    std::vector<double> ph((size_t)g.h * d.L * 2);
    for (int j = 0; j < g.h; ++j)
      for (int m = 0; m < d.L; ++m) {
        const long double ang = (long double)m * (long double)g.ring_phi0[j];
        ph[((size_t)j * d.L + m) * 2] = (double)cosl(ang);
        ph[((size_t)j * d.L + m) * 2 + 1] = (double)sinl(ang);
      }
    shot_status st2;
    // the row kernel holds two buffers and the twiddles of nbuf entries in
    // LDS: where Bluestein's buffers would not fit (float64 at Nside 512),
    // every ring keeps its direct stages
    if ((size_t)3 * nbuf * (f64 ? 16 : 8) > 160 * 1024) {
      for (auto& R : rings) R.bm = 0;
      nbuf = d.nlon;
    }
    if (blu.empty()) blu.assign(2, 0.0);
    g.ring_nbuf = nbuf;
    if ((st2 = upload((void**)&g.d_ring, rings, s)) != SHOT_OK) return st2;
    // Row workgroups take ring pairs in an XCD-contiguous order by default, so
    // the polar caps' long-prime rings (Bluestein convolutions) pile up on a
    // few XCDs (Nside 256: 1.8x the mean FFT work on one, 0.15x on another).
    // Deal them instead in octets of neighbouring pairs (which share the
    // spectrum's cache lines in an XCD's L2), eight octets per XCD, balanced
    // by a work model: n times the sum of the radices (radix-2 to 5 stages
    // counted as 2), or two power-of-two FFTs of length M for a Bluestein ring.
    if (g.h % 64 == 0) {
      auto ring_work = [](const RingDev& R) {
        if (R.bm > 0) return 2.0 * R.bm * std::log2((double)R.bm) + 4.0 * R.bm;
        double w = 0.0;
        for (int k = 0; k < R.nfac; ++k) w += R.fac[k] > 5 ? R.fac[k] : 2;
        return (double)R.len * w;
      };
      const int noct = g.h / 8;
      std::vector<int> oct_w(noct, 0);
      for (int j = 0; j < g.h; ++j) oct_w[j / 8] += (int)std::lround(ring_work(rings[j]));
      const std::vector<int> oord = balanced_dispatch(oct_w, 8, 1.0);  // oord[r * 8 + x]: round r of XCD x
      std::vector<int> rpair(g.h);
      for (int b = 0; b < g.h; ++b) {
        const int x = b & 7, k = b >> 3;  // workgroup b runs on XCD x as its k-th workgroup
        rpair[b] = oord[(k / 8) * 8 + x] * 8 + k % 8;  // octet of round k / 8 on XCD x
      }
      if ((st2 = upload((void**)&g.d_rpair, rpair, s)) != SHOT_OK) return st2;
    }
    if (f64) {
      if ((st2 = upload(&g.d_ring_tw, rtw, s)) != SHOT_OK) return st2;
      if ((st2 = upload(&g.d_ring_ph, ph, s)) != SHOT_OK) return st2;
      if ((st2 = upload(&g.d_ring_blu, blu, s)) != SHOT_OK) return st2;
    } else {
      std::vector<float> a(rtw.begin(), rtw.end()), b(ph.begin(), ph.end()), c(blu.begin(), blu.end());
      if ((st2 = upload(&g.d_ring_tw, a, s)) != SHOT_OK) return st2;
      if ((st2 = upload(&g.d_ring_ph, b, s)) != SHOT_OK) return st2;
      if ((st2 = upload(&g.d_ring_blu, c, s)) != SHOT_OK) return st2;
    }
  }
  std::vector<double> tw(2 * (size_t)d.nlon);
  for (int k = 0; k < d.nlon; ++k) {
    // exp(-2 pi i k/N), argument reduced to [0, pi/2] style accuracy by long double
    const long double ang = -2.0L * (long double)M_PI * (long double)k / (long double)d.nlon;
    tw[2 * k] = (double)cosl(ang);
    tw[2 * k + 1] = (double)sinl(ang);
  }
  shot_status st;
  if (f64) {
    if ((st = upload(&g.d_aw, aw, s)) != SHOT_OK) return st;
    if ((st = upload(&g.d_tw, tw, s)) != SHOT_OK) return st;
  } else {
    std::vector<float> awf(aw.begin(), aw.end()), twf(tw.begin(), tw.end());
    if ((st = upload(&g.d_aw, awf, s)) != SHOT_OK) return st;
    if ((st = upload(&g.d_tw, twf, s)) != SHOT_OK) return st;
  }
  // Legendre data
  std::vector<double> xs(g.x.begin(), g.x.begin() + g.h);
  int mode = leg_mode;
  if (mode == SHOT_LEG_AUTO) mode = P->prec == SHOT_BF16X3_MFMA ? SHOT_LEG_RECURRENCE : SHOT_LEG_TABLE;
  if (mode == SHOT_LEG_TABLE) {
    std::vector<double> tab;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    legendre_rows(d.L, xs, g.hpad, tab, (int)hw);
    if (P->prec == SHOT_FP64) {
      g.tab_kind = TAB_F64;
      st = upload(&g.d_tab, tab, s);
    } else if (P->prec == SHOT_FP32) {
      g.tab_kind = TAB_F32;
      std::vector<float> t32(tab.begin(), tab.end());
      st = upload(&g.d_tab, t32, s);
    } else {
      g.tab_kind = TAB_BF16;
      std::vector<uint16_t> t16(tab.size());
      for (size_t i = 0; i < tab.size(); ++i) t16[i] = to_bf16(tab[i]);
      st = upload(&g.d_tab, t16, s);
    }
    if (st != SHOT_OK) return st;
    if (mma_table(g)) {
      // the MFMA kernel runs one order per workgroup column: deal the orders
      // so that the rows meeting on one compute unit add up evenly
      std::vector<int> rows(d.L);
      for (int m = 0; m < d.L; ++m) rows[m] = d.L - m;
      // (streaming the table, two workgroups per unit keep up: factor 1, which
      // measured 4048 -> 4104 iterations/s for one bf16 item against 0.95)
      if ((st = upload((void**)&g.d_morder, balanced_dispatch(rows, 256, 1.0), s)) != SHOT_OK) return st;
    }
  } else {
    g.tab_kind = TAB_RECUR;
    std::vector<double> coef, gam, seed;
    legendre_recurrence_data(d.L, xs, coef, gam, seed);
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    // Row-split work lists: whole orders, and, for grids whose longest order
    // does not fit the kernel's LDS, orders cut into the longest parts that do.
    int part_rows = (d.L + 63) / 64 * 64;
    while (part_rows > 64 && split_lds_bytes(part_rows, g.h, 1, f64 ? 8 : 4) > 60 * 1024) part_rows -= 64;
    for (int k = 0; k < 2; ++k) {
      SplitSched& S = k ? g.ss : g.sw;
      std::vector<SplitPartH> parts;
      std::vector<double> ck;
      S.npb = split_schedule(d.L, k ? part_rows : 0, parts);
      if (k && S.npb == 0) break;  // no order is longer than a part
      S.n = (int)parts.size();
      S.maxlen = 0;
      for (const auto& q : parts) S.maxlen = std::max(S.maxlen, q.r_hi - q.r_lo);
      // dispatch order: rows balanced over the 256 compute units.  The list is
      // stored in that order (workgroup b runs entry b; the partial-buffer slots
      // travel inside the entries), so a workgroup reads its entry with one load
      // instead of an index load followed by a dependent entry load.
      std::vector<int> wts;
      // weight = rows + 64: a workgroup's fixed cost (prologue, combine, store)
      // in rows (interleaved timings at L = 720: +0 10163, +32 10203, +64
      // 10223 iterations/s)
      for (const auto& q : parts) wts.push_back(q.r_hi - q.r_lo + 64);
      const std::vector<int> order = balanced_dispatch(wts, 256);
      std::vector<SplitPartH> run(parts.size());
      for (size_t b = 0; b < order.size(); ++b) run[b] = parts[order[b]];
      legendre_checkpoints(d.L, xs, coef, seed, run, ck, (int)hw);
      if ((st = upload((void**)&S.d_parts, run, s)) != SHOT_OK) return st;
      if ((st = upload((void**)&S.d_ck, ck, s)) != SHOT_OK) return st;
      if (k) {
        std::vector<int2> cut(d.L, make_int2(1, -1));
        for (const auto& q : parts)
          if (q.s == 0) cut[q.m] = make_int2(q.ns, q.pslot);
        if ((st = upload((void**)&g.d_cut, cut, s)) != SHOT_OK) return st;
      }
    }
    if (g.ss.n > 0) {
      const size_t pb = (size_t)4 * 2 * g.ss.npb * 2 * g.h * (f64 ? 16 : 8);
      HIP_TRY(hipMalloc(&g.d_pbuf, pb));
    }
    if ((st = upload((void**)&g.d_xs, xs, s)) != SHOT_OK) return st;
    // (the matrix-core recurrence kernel reads up to 32 coefficients past an
    // order's end with wave-uniform indices: pad past the last order)
    coef.resize(coef.size() + 64, 0.0);
    if ((st = upload((void**)&g.d_rcoef, coef, s)) != SHOT_OK) return st;
    if ((st = upload((void**)&g.d_rgam, gam, s)) != SHOT_OK) return st;
    if ((st = upload((void**)&g.d_rseed, seed, s)) != SHOT_OK) return st;
  }
  return SHOT_OK;
}

// ---------------------------------------------------------------------------
// Per-call layout: items grouped by grid, with offsets into the user's arrays
// and into the plan workspace.
// ---------------------------------------------------------------------------
struct Group {
  int grid;
  int first;  // index into the sorted item list
  int count;
};

struct Layout {
  std::vector<int> order;          // sorted position -> user item index
  std::vector<int64_t> user_foff;  // by user item: field offset
  std::vector<int64_t> user_coff;  // by user item: coefficient offset
  std::vector<Group> groups;
  int64_t spec_total = 0;          // complex elements
  std::vector<int64_t> sorted_soff; // by sorted position: spectral workspace offset
  int64_t field_total = 0;         // elements
  int hs = 0, Lmax = 0;
};

shot_status make_layout(const shot_plan_s* P, const int32_t* grid_of_item, int nitems, Layout& Lo) {
  if (nitems <= 0 || !grid_of_item) return SHOT_E_INVALID;
  const int ng = (int)P->grids.size();
  Lo = Layout{};  // a layout may be rebuilt in place: every running total starts again
  Lo.user_foff.assign(nitems, 0);
  Lo.user_coff.assign(nitems, 0);
  int64_t fo = 0, co = 0;
  for (int i = 0; i < nitems; ++i) {
    const int g = grid_of_item[i];
    if (g < 0 || g >= ng) return SHOT_E_INVALID;
    Lo.user_foff[i] = fo;
    Lo.user_coff[i] = co;
    fo += P->grids[g].n();
    const int64_t L = P->grids[g].d.L;
    co += L * (L + 1) / 2;
    Lo.hs = std::max(Lo.hs, P->grids[g].h);
    Lo.Lmax = std::max<int>(Lo.Lmax, (int)L);
  }
  Lo.field_total = fo;
  Lo.order.resize(nitems);
  std::iota(Lo.order.begin(), Lo.order.end(), 0);
  std::stable_sort(Lo.order.begin(), Lo.order.end(),
                   [&](int a, int b) { return grid_of_item[a] < grid_of_item[b]; });
  Lo.groups.clear();
  Lo.sorted_soff.assign(nitems, 0);
  for (int s = 0; s < nitems; ++s) {
    const int g = grid_of_item[Lo.order[s]];
    if (Lo.groups.empty() || Lo.groups.back().grid != g) Lo.groups.push_back({g, s, 0});
    Lo.groups.back().count++;
    Lo.sorted_soff[s] = Lo.spec_total;  // the same running sum as the item descriptors' soff
    Lo.spec_total += 2LL * P->grids[g].d.L * P->grids[g].h;
  }
  return SHOT_OK;
}

// Workspace carve-out for one call.
template <typename T>
struct Work {
  ItemDev* items = nullptr;
  cpx<T>* spec = nullptr;
  T* hl = nullptr;
  T* ubuf[2] = {nullptr, nullptr};
  T* vbuf[2] = {nullptr, nullptr};
  double* red = nullptr;
  double* rhist = nullptr;
  double* prep = nullptr;
  double* res = nullptr;
  double* ehist = nullptr;
  int* brk = nullptr;
  double* kr = nullptr;
  int nslot = 0;
};

// fixed_base != nullptr: carve from that device buffer of fixed_cap bytes
// (the no-allocation entry point's scratch) instead of the plan's arena.
template <typename T>
shot_status carve(shot_plan_s* P, const Layout& Lo, int nitems, bool sinkhorn, int nslot, Work<T>& W,
                  char* fixed_base = nullptr, size_t fixed_cap = 0) {
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  const size_t o_items = take(sizeof(ItemDev) * nitems);
  const size_t o_spec = take(sizeof(cpx<T>) * Lo.spec_total);
  // (+ 32 entries: the row-split Legendre kernel prefetches up to 15 rows past an order's end)
  const size_t o_hl = take(sizeof(T) * ((size_t)nitems * Lo.Lmax + 32));
  size_t o_u0 = 0, o_u1 = 0, o_v0 = 0, o_v1 = 0, o_red = 0, o_rh = 0, o_prep = 0, o_res = 0, o_eh = 0, o_brk = 0,
         o_kr = 0;
  if (sinkhorn) {
    o_u0 = take(sizeof(T) * Lo.field_total);
    o_u1 = take(sizeof(T) * Lo.field_total);
    o_v0 = take(sizeof(T) * Lo.field_total);
    o_v1 = take(sizeof(T) * Lo.field_total);
    o_red = take(sizeof(double) * 2 * (size_t)nitems * Lo.hs * RED_SLOTS);
    o_rh = take(sizeof(double) * (size_t)nitems * nslot * Lo.hs);
    o_prep = take(sizeof(double) * (size_t)nitems * Lo.hs * 4);
    o_res = take(sizeof(double) * (size_t)nitems * 8);
    o_eh = take(sizeof(double) * (size_t)nitems * nslot);
    o_brk = take(sizeof(int) * (size_t)nitems);
    o_kr = take(sizeof(double) * (size_t)nitems);
  }
  char* b = fixed_base;
  if (b) {
    if (off > fixed_cap) {
      snprintf(g_last_error, sizeof(g_last_error),
               "call needs %zu bytes of workspace, the no-allocation scratch holds %zu", off, fixed_cap);
      return SHOT_E_INVALID;
    }
  } else {
    shot_status st = grow(P->ws, off);
    if (st != SHOT_OK) return st;
    b = static_cast<char*>(P->ws.p);
  }
  W.items = reinterpret_cast<ItemDev*>(b + o_items);
  W.spec = reinterpret_cast<cpx<T>*>(b + o_spec);
  W.hl = reinterpret_cast<T*>(b + o_hl);
  if (sinkhorn) {
    W.ubuf[0] = reinterpret_cast<T*>(b + o_u0);
    W.ubuf[1] = reinterpret_cast<T*>(b + o_u1);
    W.vbuf[0] = reinterpret_cast<T*>(b + o_v0);
    W.vbuf[1] = reinterpret_cast<T*>(b + o_v1);
    W.red = reinterpret_cast<double*>(b + o_red);
    W.rhist = reinterpret_cast<double*>(b + o_rh);
    W.prep = reinterpret_cast<double*>(b + o_prep);
    W.res = reinterpret_cast<double*>(b + o_res);
    W.ehist = reinterpret_cast<double*>(b + o_eh);
    W.brk = reinterpret_cast<int*>(b + o_brk);
    W.kr = reinterpret_cast<double*>(b + o_kr);
    W.nslot = nslot;
  }
  return SHOT_OK;
}

// Per-call status arrays: no breakdown yet, kernel ratio +inf.
template <typename T>
shot_status init_status(Work<T>& W, int nitems, hipStream_t s) {
  std::vector<int> brk0(nitems, INT_MAX);
  std::vector<double> kr0(nitems, INFINITY);
  HIP_TRY(hipMemcpyAsync(W.brk, brk0.data(), sizeof(int) * nitems, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(W.kr, kr0.data(), sizeof(double) * nitems, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return SHOT_OK;
}

// Host-side item descriptors and heat multipliers (sorted order).
template <typename T>
shot_status upload_items(shot_plan_s* P, const Layout& Lo, const int32_t* grid_of_item,
                         const std::vector<double>& eps, const std::vector<double>& tau,
                         const std::vector<double>& tvals, const std::vector<const void*>& pp,
                         const std::vector<const void*>& qq, Work<T>& W, hipStream_t s) {
  const int nitems = (int)Lo.order.size();
  std::vector<ItemDev> items(nitems);
  std::vector<T> hl((size_t)nitems * Lo.Lmax, (T)0);
  int64_t soff = 0;
  for (int si = 0; si < nitems; ++si) {
    const int ui = Lo.order[si];
    const GridRec& g = P->grids[grid_of_item[ui]];
    ItemDev& I = items[si];
    I.foff = Lo.user_foff[ui];
    I.soff = soff;
    I.coff = Lo.user_coff[ui];
    soff += 2LL * g.d.L * g.h;
    // kernels index p and q with the item's field offset: pre-subtract it, so
    // that an item's marginals may live anywhere (the divergence aliases them)
    I.p = pp.empty() ? nullptr : static_cast<const T*>(pp[ui]) - I.foff;
    I.q = qq.empty() ? nullptr : static_cast<const T*>(qq[ui]) - I.foff;
    I.eps = eps.empty() ? 0.0 : eps[ui];
    I.tau = tau.empty() ? INFINITY : tau[ui];
    I.balanced = std::isinf(I.tau) ? 1 : 0;
    I.lam = I.balanced ? 1.0 : I.tau / (I.tau + I.eps);
    I.eot = I.balanced ? 0.0 : I.eps / I.tau;
    I.pad = 0;
    const double t = tvals[ui];
    for (int l = 0; l < g.d.L; ++l) hl[(size_t)si * Lo.Lmax + l] = (T)std::exp(-t * l * (l + 1.0));
  }
  HIP_TRY(hipMemcpyAsync(W.items, items.data(), sizeof(ItemDev) * nitems, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(W.hl, hl.data(), sizeof(T) * hl.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));  // host staging vectors go out of scope
  return SHOT_OK;
}

const SplitSched* leg_split(const shot_plan_s* P, const GridRec& g, int nb, int leg_mode, int* ib_out);

// leg_mode: mode of the Legendre launch whose spectrum a row launch reads
// (it decides which kernel ran, and so whether long orders arrive in parts).
template <typename T>
RowArgs<T> row_args(const shot_plan_s* P, const GridRec& g, const Layout& Lo, const Group& G, const Work<T>& W,
                    int nitems, int leg_mode = 0) {
  RowArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.store_field = 1;
  int cib = 1;
  if (leg_split(P, g, G.count, leg_mode, &cib) == &g.ss) {  // spectra arrive with long orders in parts
    a.cut = g.d_cut;
    a.pbuf = g.d_pbuf;
    a.npb = g.ss.npb;
    a.cut_ib = cib;
  }
  a.nlat = g.d.nlat;
  a.nlon = g.d.nlon;
  a.L = g.d.L;
  a.h = g.h;
  a.hs = Lo.hs;
  a.nfac = (int)g.fac.size();
  for (int i = 0; i < a.nfac && i < 8; ++i) a.fac[i] = g.fac[i];
  a.tw = static_cast<const cpx<T>*>(g.d_tw);
  a.aw = static_cast<const T*>(g.d_aw);
  if (g.hp) {
    a.ring = g.d_ring;
    // the dealt order pays when workgroups outnumber the 256 compute units (a
    // unit then runs several and their work adds up); with one workgroup per
    // unit the launch ends with its slowest group either way (measured: Nside
    // 256 one item +15 %, Nside 64 batches +8 %, Nside 64 and 128 one item -0.5 to -0.9 %)
    a.rpair = (long long)g.h * G.count > 256 ? g.d_rpair : nullptr;
    a.ring_tw = static_cast<const cpx<T>*>(g.d_ring_tw);
    a.ring_ph = static_cast<const cpx<T>*>(g.d_ring_ph);
    a.ring_blu = static_cast<const cpx<T>*>(g.d_ring_blu);
    a.nbuf = g.ring_nbuf;
  }
  a.item0 = G.first;
  a.items = W.items;
  a.spec = W.spec;
  a.ubuf0 = W.ubuf[0];
  a.ubuf1 = W.ubuf[1];
  a.vbuf0 = W.vbuf[0];
  a.vbuf1 = W.vbuf[1];
  a.red = W.red;
  a.nitems_all = nitems;
  a.rhist = W.rhist;
  a.nslot = W.nslot;
  a.chk_slot = -1;
  a.prep = W.prep;
  a.brk = W.brk;
  a.kr = W.kr;
  return a;
}

template <typename T>
LegArgs<T> leg_args(const GridRec& g, const Group& G, const Work<T>& W, int hl_stride, const Layout& Lo) {
  LegArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.soff0 = Lo.sorted_soff[G.first];
  a.L = g.d.L;
  a.h = g.h;
  a.hpad = g.hpad;
  a.tab = g.d_tab;
  a.morder = g.d_morder;
  a.xs = g.d_xs;
  a.rcoef = g.d_rcoef;
  a.rgam = g.d_rgam;
  a.rseed = g.d_rseed;
  a.item0 = G.first;
  a.nb = G.count;
  a.items = W.items;
  a.spec = W.spec;
  a.hl = W.hl;
  a.hl_stride = hl_stride;
  a.mode = 0;
  a.jpt = g.tune_jpt;
  return a;
}

// Items per Legendre workgroup: as many as requested/available, capped so the
// LDS staging (inputs IB*2h + coefficients IB*L complex) stays within 64 KiB.
int pick_ib(const shot_plan_s* P, const GridRec& g, int count) {
  int ib = g.tune_ib > 0 ? g.tune_ib : (P->leg_ib > 0 ? P->leg_ib : 8);
  while (ib > 1 && ib > count) ib >>= 1;
  if (g.tab_kind == TAB_RECUR) {
    // coefficients (2 doubles) and IB double2 inputs per row, padded to 16 rows
    const size_t npad = (g.d.L + 15) / 16 * 16;
    ib = std::min(ib, 4);
    while (ib > 1 && npad * 16 * (1 + ib) > 56 * 1024) ib >>= 1;
    return ib;
  }
  const size_t cs = P->prec == SHOT_FP64 ? 16 : 8;
  while (ib > 1 && (size_t)ib * (2 * g.h + g.d.L) * cs > 60 * 1024) ib >>= 1;
  return ib;
}

// Row-split work list for a launch of nb items, ib per workgroup: whole
// orders, or orders cut into parts when only the cut list fits in LDS (at most
// 4 chunks: the partial buffer is sized for that); nullptr when neither fits.
const SplitSched* pick_sched(const shot_plan_s* P, const GridRec& g, int nb, int ib) {
  const int rb = P->prec == SHOT_FP64 ? 8 : 4;
  const int chunks = (nb + ib - 1) / ib;
  const bool cut_ok = g.ss.n > 0 && chunks <= 4 && split_lds_bytes(g.ss.maxlen, g.h, ib, rb) <= 60 * 1024;
  const bool whole_ok = g.sw.n > 0 && split_lds_bytes(g.sw.maxlen, g.h, ib, rb) <= 60 * 1024;
  if (cut_ok && !whole_ok) return &g.ss;
  return whole_ok ? &g.sw : nullptr;
}

// Row-split recurrence kernel: used unless a chains-per-thread tuning selects
// the latitude-split kernel, when ceil(nlat/2) <= 512 and its LDS fits.
bool use_split(const shot_plan_s* P, const GridRec& g) {
  if (g.tab_kind != TAB_RECUR || g.tune_jpt != 0 || g.h > 512) return false;
  return pick_sched(P, g, 1, 1) != nullptr;
}

// Matrix-core kernel for table grids: column tiles per workgroup, or 0 for
// the VALU kernels.  Automatic: matrix cores from 4 items on, the widest tile
// count (<= the batch) whose LDS staging fits.
int mma_tiles(const shot_plan_s* P, const GridRec& g, int count) {
  if (!mma_table(g) || g.tune_jpt < 0) return 0;
  int nt = g.tune_jpt;
  // Matrix cores for any item count: they stream the table faster than the
  // VALU table kernel even for a single item (one item at L = 720: bf16
  // 0.58 -> 0.12 ms per launch, fp32 0.80 -> 0.53 ms)
  if (nt == 0) nt = count >= 32 ? 4 : (count >= 16 ? 2 : 1);
  // fewer column tiles while they overflow 60 KiB of LDS (several workgroups
  // per compute unit); one tile may take up to 150 KiB (fp32 tables of long
  // orders, one workgroup per unit)
  while (nt > 1 && mma_lds_bytes(g.d.L, g.hpad, nt, g.tab_kind) > 60 * 1024) nt >>= 1;
  if (mma_lds_bytes(g.d.L, g.hpad, nt, g.tab_kind) > 150 * 1024) return 0;
  (void)P;
  return nt;
}

// Recurrence-fed matrix-core kernel for a fused (mode 0) launch of `count`
// items: column tiles per workgroup (1 or 2, i.e. 8 or 16 items), or 0 for
// the VALU kernels; *op_out gets the operand form of the plan's precision.
// bfloat16 and split-bfloat16 plans always take it (their precision is that of
// the operands); float32 plans when tuned to 8 or 16 items per workgroup.
int rmma_tiles(const shot_plan_s* P, const GridRec& g, int count, int leg_mode, int* op_out) {
  if (leg_mode != 0 || g.tab_kind != TAB_RECUR || P->prec == SHOT_FP64 || g.hp || g.h > 512) return 0;
  const int op = P->prec == SHOT_FP32 ? RM_F32 : (P->prec == SHOT_BF16_MFMA ? RM_BF16 : RM_BF16X3);
  int nt;
  if (g.tune_ib >= 8) nt = g.tune_ib / 8;
  else if (P->prec == SHOT_FP32) return 0;
  else nt = 1;  // one column tile: two workgroups fit a compute unit's LDS
  while (nt > 1 && rmma_lds_bytes(g.d.L, g.h, nt, op) > 160 * 1024) nt >>= 1;
  if (rmma_lds_bytes(g.d.L, g.h, nt, op) > 160 * 1024) return 0;
  if (op_out) *op_out = op;
  return nt;
}

int split_ib(const shot_plan_s* P, const GridRec& g, int count) {
  int ib = (g.tune_ib == 2 || (g.tune_ib == 0 && count >= 2)) ? 2 : 1;
  if (ib == 2 && (g.h > 384 || !pick_sched(P, g, count, 2))) ib = 1;  // 2 items: at most 6 chains per lane
  return ib;
}

template <typename T>
shot_status run_rows(shot_plan_s* P, const RowArgs<T>& a, int nb, hipStream_t s) {
  ProfScope ps(P, s, 1);
  hipError_t e = launch_rows<T>(a, nb, s);
  return e == hipSuccess ? SHOT_OK : hip_fail(e, "row kernel launch", __LINE__);
}

// Row-split work list of a Legendre launch of nb items (nullptr when another
// kernel runs it) and its items per workgroup.
const SplitSched* leg_split(const shot_plan_s* P, const GridRec& g, int nb, int leg_mode, int* ib_out) {
  if (mma_tiles(P, g, nb) > 0 || rmma_tiles(P, g, nb, leg_mode, nullptr) > 0 || !use_split(P, g)) return nullptr;
  const int ib = split_ib(P, g, nb);
  if (ib_out) *ib_out = ib;
  return pick_sched(P, g, nb, ib);
}

template <typename T>
shot_status run_leg(shot_plan_s* P, const GridRec& g, LegArgs<T> a, hipStream_t s) {
  ProfScope ps(P, s, 0);
  hipError_t e;
  int ib = 1, op = 0;
  const int nt = mma_tiles(P, g, a.nb);
  const int rnt = rmma_tiles(P, g, a.nb, a.mode, &op);
  if (nt > 0) {
    e = launch_legendre_mma<T>(a, g.tab_kind, nt, s);
  } else if (rnt > 0) {
    e = launch_legendre_rmma<T>(a, op, rnt, s);
  } else if (const SplitSched* S = leg_split(P, g, a.nb, a.mode, &ib)) {
    a.parts = S->d_parts;
    a.nparts = S->n;
    a.maxlen = S->maxlen;
    a.rck = S->d_ck;
    a.npb = S->npb;
    a.pbuf = g.d_pbuf;
    e = launch_legendre_split<T>(a, ib, s);
  } else {
    const int ib = pick_ib(P, g, a.nb);
    e = launch_legendre<T>(a, g.tab_kind, ib, s);
  }
  return e == hipSuccess ? SHOT_OK : hip_fail(e, "Legendre kernel launch", __LINE__);
}

#define ST_TRY(expr)                     \
  do {                                   \
    shot_status s_ = (expr);             \
    if (s_ != SHOT_OK) return s_;        \
  } while (0)

// ---------------------------------------------------------------------------
// Heat apply / analysis / synthesis
// ---------------------------------------------------------------------------
template <typename T>
shot_status heat_apply_impl(shot_plan_s* P, const int32_t* goi, int nitems, const double* t,
                            const void* v, void* out, int transpose, hipStream_t s,
                            char* fixed_base = nullptr, size_t fixed_cap = 0) {
  Layout Lo;
  ST_TRY(make_layout(P, goi, nitems, Lo));
  Work<T> W;
  ST_TRY(carve<T>(P, Lo, nitems, false, 0, W, fixed_base, fixed_cap));
  std::vector<double> tv(t, t + nitems);
  ST_TRY(upload_items<T>(P, Lo, goi, {}, {}, tv, {}, {}, W, s));
  for (const Group& G : Lo.groups) {
    const GridRec& g = P->grids[G.grid];
    RowArgs<T> a = row_args<T>(P, g, Lo, G, W, nitems);
    a.mode = ROW_FWD;
    a.in = static_cast<const T*>(v);
    a.wts_in = transpose ? 0 : 1;
    ST_TRY(run_rows<T>(P, a, G.count, s));
    ST_TRY(run_leg<T>(P, g, leg_args<T>(g, G, W, Lo.Lmax, Lo), s));
    a.mode = ROW_INV;
    a.out = static_cast<T*>(out);
    a.wts_out = transpose ? 1 : 0;
    ST_TRY(run_rows<T>(P, a, G.count, s));
  }
  return SHOT_OK;
}

template <typename T>
shot_status sht_impl(shot_plan_s* P, const int32_t* goi, int nitems, const void* in, void* out,
                     bool analysis, hipStream_t s) {
  Layout Lo;
  ST_TRY(make_layout(P, goi, nitems, Lo));
  Work<T> W;
  ST_TRY(carve<T>(P, Lo, nitems, false, 0, W));
  std::vector<double> tv(nitems, 0.0);
  ST_TRY(upload_items<T>(P, Lo, goi, {}, {}, tv, {}, {}, W, s));
  for (const Group& G : Lo.groups) {
    const GridRec& g = P->grids[G.grid];
    RowArgs<T> a = row_args<T>(P, g, Lo, G, W, nitems, analysis ? 1 : 2);
    LegArgs<T> la = leg_args<T>(g, G, W, Lo.Lmax, Lo);
    if (analysis) {
      a.mode = ROW_FWD;
      a.in = static_cast<const T*>(in);
      a.wts_in = 1;
      ST_TRY(run_rows<T>(P, a, G.count, s));
      la.mode = 1;
      la.coeff = static_cast<cpx<T>*>(out);
      ST_TRY(run_leg<T>(P, g, la, s));
    } else {
      la.mode = 2;
      la.coeff = static_cast<cpx<T>*>(const_cast<void*>(in));
      ST_TRY(run_leg<T>(P, g, la, s));
      a.mode = ROW_INV;
      a.out = static_cast<T*>(out);
      ST_TRY(run_rows<T>(P, a, G.count, s));
    }
  }
  return SHOT_OK;
}

// ---------------------------------------------------------------------------
// Sinkhorn solve on items described by per-item (p, q) device pointers.
// ---------------------------------------------------------------------------
struct SolveSpec {
  std::vector<int32_t> grid;       // per item
  std::vector<shot_params> prm;    // per item
  std::vector<const void*> p, q;   // per item device pointers
};

shot_status check_params(const shot_params& pr) {
  if (!(pr.eps > 0) || !std::isfinite(pr.eps)) return SHOT_E_INVALID;
  if (!(pr.tau > 0)) return SHOT_E_INVALID;
  if (pr.max_iter < 1 || pr.check_every < 1 || !(pr.tol >= 0)) return SHOT_E_INVALID;
  return SHOT_OK;
}

template <typename T>
shot_status finish_solve(shot_plan_s* P, const Layout& Lo, Work<T>& W, int nitems, int K, int C,
                         int final_slot, double tol, T* phi, T* psi, shot_solve_info* info,
                         double* mass_out, hipStream_t s, T* u_last = nullptr, T* v_last = nullptr);

// Whether the reverse sweep over these fields keeps the whole forward history:
// 2 T fields per item within half the free device memory and 64 GiB.
template <typename T>
bool whole_history_fits(long long field_total, int T_iter) {
  size_t fr = 0, tot = 0;
  const double hist = 2.0 * sizeof(T) * (double)field_total * T_iter;
  return hipMemGetInfo(&fr, &tot) == hipSuccess && hist <= std::min(0.5 * (double)fr, 64.0 * 1024 * 1024 * 1024);
}

template <typename T>
shot_status solve_impl(shot_plan_s* P, const SolveSpec& S, T* phi, T* psi, shot_solve_info* info,
                       double* mass_out, hipStream_t s) {
  const int nitems = (int)S.grid.size();
  Layout Lo;
  ST_TRY(make_layout(P, S.grid.data(), nitems, Lo));
  int T_iter = 0, C = S.prm[0].check_every;
  double tol = S.prm[0].tol;
  for (int i = 0; i < nitems; ++i) {
    ST_TRY(check_params(S.prm[i]));
    T_iter = std::max(T_iter, S.prm[i].max_iter);
    if (S.prm[i].check_every != C || S.prm[i].tol != tol || S.prm[i].max_iter != S.prm[0].max_iter)
      return SHOT_E_UNSUPPORTED;  // one call advances all items in lock step
  }
  const int nchk = T_iter / C;
  const int nslot = nchk + 1;  // + final residual
  Work<T> W;
  ST_TRY(carve<T>(P, Lo, nitems, true, nslot, W));
  std::vector<double> eps(nitems), tau(nitems), tv(nitems);
  for (int i = 0; i < nitems; ++i) {
    eps[i] = S.prm[i].eps;
    tau[i] = S.prm[i].tau;
    tv[i] = S.prm[i].eps / 4.0;  // t = eps/4 (Alg. 1)
  }
  ST_TRY(upload_items<T>(P, Lo, S.grid.data(), eps, tau, tv, S.p, S.q, W, s));
  ST_TRY(init_status(W, nitems, s));

  auto each_group = [&](auto&& fn) -> shot_status {
    for (const Group& G : Lo.groups) {
      shot_status st = fn(G, P->grids[G.grid]);
      if (st != SHOT_OK) return st;
    }
    return SHOT_OK;
  };
  hipStream_t ls = s;  // launch stream (the capture stream while recording a graph)
  auto rows = [&](const Group& G, const GridRec& g, int mode, int k, int chk) {
    RowArgs<T> a = row_args<T>(P, g, Lo, G, W, nitems);
    a.mode = mode;
    a.k = k;
    a.chk_slot = chk;
    a.out = phi;
    a.out2 = psi;
    // u_k is read again only by the next half-iteration's check (k a check
    // iteration), by the closing residual and by the potentials (k = T, or a
    // check iteration where an early stop may land); v_k only by the
    // potentials
    if (mode == ROW_SINK_U || mode == ROW_SINK_V) a.store_field = (k % C == 0 || k == T_iter) ? 1 : 0;
    return run_rows<T>(P, a, G.count, ls);
  };
  auto leg = [&](const Group& G, const GridRec& g) { return run_leg<T>(P, g, leg_args<T>(g, G, W, Lo.Lmax, Lo), ls); };

  int K = T_iter;
  int final_slot = nslot - 1;
  bool early = false;
  if (K % C == 0) final_slot = K / C - 1;
  // Fixed T: the launch sequence depends only on the layout, so it is recorded
  // once as a HIP graph (per-call data lives in device memory) and replayed.
  auto fixed_loop = [&]() -> shot_status {
    ST_TRY(each_group([&](const Group& G, const GridRec& g) { return rows(G, g, ROW_INIT, 0, -1); }));
    for (int k = 1; k <= T_iter; ++k) {
      const bool chk_prev = (k - 1 >= 1) && ((k - 1) % C == 0);
      const int slot = chk_prev ? (k - 1) / C - 1 : -1;
      ST_TRY(each_group([&](const Group& G, const GridRec& g) {
        shot_status st = leg(G, g);
        return st != SHOT_OK ? st : rows(G, g, ROW_SINK_U, k, slot);
      }));
      ST_TRY(each_group([&](const Group& G, const GridRec& g) {
        shot_status st = leg(G, g);
        return st != SHOT_OK ? st : rows(G, g, ROW_SINK_V, k, -1);
      }));
    }
    return each_group([&](const Group& G, const GridRec& g) {
      shot_status st = leg(G, g);
      return st != SHOT_OK ? st : rows(G, g, ROW_CHECK, K + 1, final_slot);
    });
  };
  // Under capture, the grid groups of a call touch disjoint items: each group's
  // whole loop is recorded on its own branch (the first on the capture stream,
  // the others on side streams forked from it and joined back), so that the
  // replayed graph can run the groups side by side.
  auto fixed_loop_branches = [&]() -> shot_status {
    const int ng = (int)Lo.groups.size();
    if (ng == 1) return fixed_loop();
    while ((int)P->branch.size() < ng - 1) {
      hipStream_t b = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
      P->branch.push_back(b);
    }
    while ((int)P->bev.size() < ng) {
      hipEvent_t e = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      P->bev.push_back(e);
    }
    hipStream_t cs = ls;
    HIP_TRY(hipEventRecord(P->bev[0], cs));
    for (int gi = 0; gi < ng; ++gi) {
      const Group& G = Lo.groups[gi];
      const GridRec& g = P->grids[G.grid];
      ls = gi == 0 ? cs : P->branch[gi - 1];
      if (gi > 0) HIP_TRY(hipStreamWaitEvent(ls, P->bev[0], 0));
      ST_TRY(rows(G, g, ROW_INIT, 0, -1));
      for (int k = 1; k <= T_iter; ++k) {
        const bool chk_prev = (k - 1 >= 1) && ((k - 1) % C == 0);
        const int slot = chk_prev ? (k - 1) / C - 1 : -1;
        ST_TRY(leg(G, g));
        ST_TRY(rows(G, g, ROW_SINK_U, k, slot));
        ST_TRY(leg(G, g));
        ST_TRY(rows(G, g, ROW_SINK_V, k, -1));
      }
      ST_TRY(leg(G, g));
      ST_TRY(rows(G, g, ROW_CHECK, K + 1, final_slot));
    }
    for (int gi = 1; gi < ng; ++gi) {
      HIP_TRY(hipEventRecord(P->bev[gi], P->branch[gi - 1]));
      HIP_TRY(hipStreamWaitEvent(cs, P->bev[gi], 0));
    }
    ls = cs;
    return SHOT_OK;
  };
  // (event timing needs eager launches: events recorded inside a graph cannot be timed)
  if (tol == 0 && P->graphs && !P->prof) {
    std::vector<long long> key = {(long long)(uintptr_t)P->ws.p, (long long)P->ws.bytes, nitems, T_iter, C,
                                  Lo.hs, Lo.Lmax, P->prof ? 1 : 0};
    for (const Group& G : Lo.groups) {
      key.push_back(G.grid);
      key.push_back(G.first);
      key.push_back(G.count);
      key.push_back(P->grids[G.grid].tune_ib);
      key.push_back(P->grids[G.grid].tune_jpt);
    }
    if (!P->gexec || key != P->gkey) {
      drop_graph(P);
      if (!P->cap) HIP_TRY(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed));
      ls = P->cap;
      shot_status st = fixed_loop_branches();
      ls = s;
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(P->cap, &graph);
      if (st != SHOT_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != SHOT_OK ? st : hip_fail(e, "hipStreamEndCapture", __LINE__);
      }
      e = hipGraphInstantiate(&P->gexec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        P->gexec = nullptr;
        return hip_fail(e, "hipGraphInstantiate", __LINE__);
      }
      P->graph = graph;
      P->gkey = key;
    }
    HIP_TRY(hipGraphLaunch(P->gexec, s));
    return finish_solve<T>(P, Lo, W, nitems, K, C, final_slot, tol, phi, psi, info, mass_out, s);
  }

  // v_0 = 1: spectrum of the constant field, plus norms and masses
  ST_TRY(each_group([&](const Group& G, const GridRec& g) { return rows(G, g, ROW_INIT, 0, -1); }));
  final_slot = nslot - 1;
  for (int k = 1; k <= T_iter; ++k) {
    const bool chk_prev = (k - 1 >= 1) && ((k - 1) % C == 0);
    const int slot = chk_prev ? (k - 1) / C - 1 : -1;
    ST_TRY(each_group([&](const Group& G, const GridRec& g) {
      shot_status st = leg(G, g);
      return st != SHOT_OK ? st : rows(G, g, ROW_SINK_U, k, slot);
    }));
    if (tol > 0 && chk_prev) {
      // e_marg of iteration k-1 is complete: decide before the v-half
      for (const Group& G : Lo.groups) {
        RowArgs<T> a = row_args<T>(P, P->grids[G.grid], Lo, G, W, nitems);
        HIP_TRY(launch_reduce<T>(a, G.count, slot + 1, W.res, W.ehist, s));
      }
      std::vector<double> eh((size_t)nitems * nslot);
      HIP_TRY(hipMemcpyAsync(eh.data(), W.ehist, sizeof(double) * eh.size(), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      bool all = true;
      for (int si = 0; si < nitems; ++si) all &= (eh[(size_t)si * nslot + slot] < tol);
      if (all) {
        K = k - 1;
        final_slot = slot;
        early = true;
        break;
      }
    }
    ST_TRY(each_group([&](const Group& G, const GridRec& g) {
      shot_status st = leg(G, g);
      return st != SHOT_OK ? st : rows(G, g, ROW_SINK_V, k, -1);
    }));
  }
  if (!early) {
    // e_marg of the returned scalings needs K v_hat_K (one more heat apply);
    // when K is itself a check iteration its history slot is that residual
    if (K % C == 0) final_slot = K / C - 1;
    ST_TRY(each_group([&](const Group& G, const GridRec& g) {
      shot_status st = leg(G, g);
      return st != SHOT_OK ? st : rows(G, g, ROW_CHECK, K + 1, final_slot);
    }));
  }
  return finish_solve<T>(P, Lo, W, nitems, K, C, final_slot, tol, phi, psi, info, mass_out, s);
}

// Potentials, cost and reports after the iteration loop (iteration K reached).
// u_last / v_last: where the last scalings are, when not in the work buffers.
template <typename T>
shot_status finish_solve(shot_plan_s* P, const Layout& Lo, Work<T>& W, int nitems, int K, int C,
                         int final_slot, double tol, T* phi, T* psi, shot_solve_info* info,
                         double* mass_out, hipStream_t s, T* u_last, T* v_last) {
  for (const Group& G : Lo.groups) {
    RowArgs<T> a = row_args<T>(P, P->grids[G.grid], Lo, G, W, nitems);
    a.mode = ROW_FINAL;
    a.k = K;
    a.out = phi;
    a.out2 = psi;
    if (u_last) a.ubuf0 = a.ubuf1 = u_last;
    if (v_last) a.vbuf0 = a.vbuf1 = v_last;
    ST_TRY(run_rows<T>(P, a, G.count, s));
  }
  const int nchk_done = K / C;
  for (const Group& G : Lo.groups) {
    RowArgs<T> a = row_args<T>(P, P->grids[G.grid], Lo, G, W, nitems);
    a.chk_slot = final_slot;
    HIP_TRY(launch_reduce<T>(a, G.count, nchk_done, W.res, W.ehist, s));
  }
  std::vector<double> res((size_t)nitems * 8), kr(nitems);
  std::vector<int> brk(nitems);
  HIP_TRY(hipMemcpyAsync(res.data(), W.res, sizeof(double) * res.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(brk.data(), W.brk, sizeof(int) * nitems, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(kr.data(), W.kr, sizeof(double) * nitems, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int si = 0; si < nitems; ++si) {
    const int ui = Lo.order[si];
    shot_solve_info& I = info[ui];
    I.cost = res[(size_t)si * 8 + 0];
    I.err = res[(size_t)si * 8 + 1];
    I.iters = K;
    I.breakdown_iter = brk[si] == INT_MAX ? 0 : brk[si];
    I.kratio = kr[si];
    if (mass_out) {
      mass_out[2 * ui] = res[(size_t)si * 8 + 2];
      mass_out[2 * ui + 1] = res[(size_t)si * 8 + 3];
    }
    I.reserved = 0;
    // marginals must carry positive, finite area-weighted mass (Alg. 1 takes
    // measures); the masses come from the solve's own prologue reduction
    const double mp = res[(size_t)si * 8 + 2], mq = res[(size_t)si * 8 + 3];
    if (!(mp > 0) || !(mq > 0) || !std::isfinite(mp) || !std::isfinite(mq)) {
      I.status = SHOT_E_INVALID;
      snprintf(g_last_error, sizeof(g_last_error),
               "item %d: marginal masses m(p) = %g, m(q) = %g must be positive and finite", ui, mp, mq);
    } else if (I.breakdown_iter) {
      I.status = SHOT_E_BREAKDOWN;
    } else if (tol > 0 && !(I.err < tol)) {
      I.status = SHOT_W_NOT_CONVERGED;
    } else {
      I.status = SHOT_OK;
    }
  }
  return SHOT_OK;
}

// The call's status: an invalid item (an argument error) first, else the
// largest per-item code (breakdown above not-converged above ok).
shot_status worst(const shot_solve_info* info, int n) {
  int w = SHOT_OK;
  for (int i = 0; i < n; ++i) {
    if (info[i].status == SHOT_E_INVALID) return SHOT_E_INVALID;
    w = std::max(w, info[i].status);
  }
  return (shot_status)w;
}

bool ptr_ok(const void* p) { return p != nullptr; }

// Time the fused Legendre launch for each candidate (items per workgroup,
// chains per thread) on a synthetic spectrum and keep the fastest on the grid.
template <typename T>
shot_status autotune_impl(shot_plan_s* P, GridRec& g, const Layout& Lo, int nitems, hipStream_t s) {
  Work<T> W;
  ST_TRY(carve<T>(P, Lo, nitems, false, 0, W));
  std::vector<double> tv(nitems, 1e-3);
  std::vector<int32_t> goi(nitems, (int32_t)(&g - P->grids.data()));
  ST_TRY(upload_items<T>(P, Lo, goi.data(), {}, {}, tv, {}, {}, W, s));
  {
    std::vector<cpx<T>> fill((size_t)Lo.spec_total);
    for (size_t i = 0; i < fill.size(); ++i) fill[i] = {(T)(1.0 / (1.0 + (double)(i % 97))), (T)0.25};
    HIP_TRY(hipMemcpyAsync(W.spec, fill.data(), sizeof(cpx<T>) * fill.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  std::vector<std::pair<int, int>> cand;
  for (int ib : {1, 2, 4, 8}) {
    if (ib > nitems && ib != 1) continue;
    if (g.tab_kind == TAB_RECUR) {
      if (ib > 4) continue;
      if (ib <= 2) cand.push_back({ib, 0});  // row-split kernel
      for (int jpt : {1, 2, 4})
        if (recur_jpt_valid(g.h, jpt)) cand.push_back({ib, jpt});
    } else {
      cand.push_back({ib, -1});  // VALU table kernel
    }
  }
  if (mma_table(g))
    for (int nt : {1, 2, 4})
      if (16 * nt <= 2 * std::max(nitems, 8)) cand.push_back({0, nt});
  if (g.tab_kind == TAB_RECUR && P->prec != SHOT_FP64) {
    // bfloat16 and split-bfloat16 plans compute on matrix cores only
    if (P->prec != SHOT_FP32) cand.clear();
    for (int ib : {8, 16})
      if (ib <= std::max(nitems, 8)) cand.push_back({ib, 0});
  }
  const int save_ib = g.tune_ib, save_jpt = g.tune_jpt;
  const bool save_prof = P->prof;
  P->prof = false;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  std::pair<int, int> bestc = {save_ib, save_jpt};
  Group G{(int)(&g - P->grids.data()), 0, nitems};
  for (auto c : cand) {
    g.tune_ib = c.first;
    g.tune_jpt = c.second;
    if (g.tab_kind == TAB_RECUR && c.first >= 8) {
      if (rmma_tiles(P, g, nitems, 0, nullptr) != c.first / 8) continue;  // does not fit LDS
    } else if (g.tab_kind != TAB_RECUR && c.second > 0) {
      if (mma_tiles(P, g, nitems) != c.second) continue;  // does not fit LDS
    } else if (use_split(P, g) ? split_ib(P, g, nitems) != c.first : pick_ib(P, g, nitems) != c.first) {
      continue;  // does not fit LDS
    }
    if (g.tab_kind == TAB_RECUR && c.first < 8 && c.second == 0 && !use_split(P, g)) continue;
    shot_status st = SHOT_OK;
    for (int w = 0; w < 2 && st == SHOT_OK; ++w) st = run_leg<T>(P, g, leg_args<T>(g, G, W, Lo.Lmax, Lo), s);
    if (st != SHOT_OK) continue;
    (void)hipEventRecord(e0, s);
    const int reps = 5;
    for (int r = 0; r < reps && st == SHOT_OK; ++r) st = run_leg<T>(P, g, leg_args<T>(g, G, W, Lo.Lmax, Lo), s);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || st != SHOT_OK) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) { best = ms; bestc = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->prof = save_prof;
  g.tune_ib = bestc.first;
  g.tune_jpt = bestc.second;
  return SHOT_OK;
}

// Def. 2.3: S = R(p,q) - (R(p,p) + R(q,q))/2 + eps/2 (m(p) - m(q))^2, float64.
// inf holds the three solves of pair i at 3i, 3i+1, 3i+2; mass holds
// (m(first marginal), m(second marginal)) per solve.
void combine_divergence(const shot_params* prm, int npairs, const shot_solve_info* inf,
                        const double* mass, double* S) {
  for (int i = 0; i < npairs; ++i) {
    const double mp = mass[2 * (3 * i)], mq = mass[2 * (3 * i) + 1];
    const double dm = mp - mq;
    S[i] = inf[3 * i].cost - 0.5 * (inf[3 * i + 1].cost + inf[3 * i + 2].cost) + 0.5 * prm[i].eps * dm * dm;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the no-allocation heat apply.  A file-scope device array: every
// GPU the library runs on holds its own copy until the process ends.  In host
// code `scratch` names a host-side stand-in, not a device address, so host
// code only ever uses the address hipGetSymbolAddress returns for the current
// device, fetched once per device at plan creation and kept in g_scratch.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SHOT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Device `dev` must be current.
shot_status scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return SHOT_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return SHOT_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
  g_scratch[dev] = static_cast<char*>(ptr);
  return SHOT_OK;
}

char* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[dev];
}

}  // namespace

// ---------------------------------------------------------------------------
// Reverse-mode gradient of balanced Alg. 1 (see the adjoint notes in
// kernels.hip).  Items are advanced in lock step.  The forward sweep keeps
// v-hat_k and s_k every CK iterations; the reverse sweep recomputes each
// segment of CK iterations from its checkpoint (storing u-hat, v-hat and s
// for that segment only) and then walks it backwards.  Outputs p-bar and
// q-bar (gradients of each item's Alg. 1 cost with respect to its p and q).
// ---------------------------------------------------------------------------
template <typename T>
shot_status adjoint_impl(shot_plan_s* P, const SolveSpec& S, int CK, T** pbar_out, T** qbar_out,
                         Layout& Lo, hipStream_t s, shot_solve_info* fwd_info = nullptr, double* fwd_mass = nullptr,
                         int nrev = -1) {
  const int nitems = (int)S.grid.size();
  ST_TRY(make_layout(P, S.grid.data(), nitems, Lo));
  const int Tit = S.prm[0].max_iter;
  const bool unbal = !std::isinf(S.prm[0].tau);  // every item of a call takes the same branch
  for (int i = 0; i < nitems; ++i) {
    ST_TRY(check_params(S.prm[i]));
    if (std::isinf(S.prm[i].tau) == unbal || S.prm[i].tol != 0 || S.prm[i].max_iter != Tit)
      return SHOT_E_UNSUPPORTED;
  }
  // keep the whole forward history (u-hat, v-hat of every iteration) when it
  // fits: the reverse sweep then needs one forward pass instead of a
  // checkpointed pass plus a recomputation; otherwise checkpoints every
  // ceil(sqrt(T)) iterations.  With fwd_info the forward pass (which must then
  // hold the whole history) also reports each solve as solve_impl does.
  if (fwd_info) CK = Tit;
  else if (CK <= 0) CK = whole_history_fits<T>(Lo.field_total, Tit) ? Tit : (int)std::ceil(std::sqrt((double)Tit));
  CK = std::min(CK, Tit);
  const int nck = (Tit - 1) / CK;  // checkpoints at k = CK, 2CK, ... < T
  const int C = S.prm[0].check_every;
  for (int i = 0; fwd_info && i < nitems; ++i)
    if (S.prm[i].check_every != C) return SHOT_E_UNSUPPORTED;
  const int nslot = fwd_info ? Tit / C + 1 : 1;  // e_marg history, as solve_impl keeps it
  Work<T> W;
  ST_TRY(carve<T>(P, Lo, nitems, true, nslot, W));
  std::vector<double> eps(nitems), tau(nitems), tv(nitems);
  for (int i = 0; i < nitems; ++i) {
    eps[i] = S.prm[i].eps;
    tau[i] = S.prm[i].tau;
    tv[i] = S.prm[i].eps / 4.0;
  }
  ST_TRY(upload_items<T>(P, Lo, S.grid.data(), eps, tau, tv, S.p, S.q, W, s));
  ST_TRY(init_status(W, nitems, s));
  // gradient arena
  const size_t F = (size_t)Lo.field_total;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  const size_t o_specA = take(sizeof(cpx<T>) * Lo.spec_total);
  const size_t o_gA = take(sizeof(T) * F), o_gB = take(sizeof(T) * F);
  const size_t o_hu = take(sizeof(T) * F * CK), o_hv = take(sizeof(T) * F * CK);
  const size_t o_ckv = take(sizeof(T) * F * std::max(nck, 1));
  const size_t o_gh = take(sizeof(double) * nitems * (CK + 1) * 3);
  const size_t o_vbar = take(unbal ? sizeof(T) * F : 0);
  const size_t o_ckg = take(sizeof(double) * nitems * std::max(nck, 1));
  const size_t o_adjp = take(sizeof(double) * nitems * Lo.hs);
  ST_TRY(grow(P->ws2, off));
  char* b = static_cast<char*>(P->ws2.p);
  cpx<T>* specA = reinterpret_cast<cpx<T>*>(b + o_specA);
  T* gA = reinterpret_cast<T*>(b + o_gA);
  T* gB = reinterpret_cast<T*>(b + o_gB);
  T* hu = reinterpret_cast<T*>(b + o_hu);
  T* hv = reinterpret_cast<T*>(b + o_hv);
  T* ckv = reinterpret_cast<T*>(b + o_ckv);
  double* gh = reinterpret_cast<double*>(b + o_gh);
  double* ckg = reinterpret_cast<double*>(b + o_ckg);
  double* adjp = reinterpret_cast<double*>(b + o_adjp);
  T* vbar = reinterpret_cast<T*>(b + o_vbar);

  auto base_args = [&](const Group& G, const GridRec& g) {
    RowArgs<T> a = row_args<T>(P, g, Lo, G, W, nitems);
    a.gA = gA;
    a.gB = gB;
    a.adjp = adjp;
    a.kT = Tit;
    a.vbar = vbar;
    return a;
  };
  // items of each group that the reverse sweep runs: all, or (nrev >= 0) the
  // call's first nrev items, which open every group (the others, after them,
  // run forward only: their solves are reported, not differentiated)
  std::vector<int> rev_count(Lo.groups.size());
  for (size_t gi = 0; gi < Lo.groups.size(); ++gi) {
    const Group& G = Lo.groups[gi];
    int n = 0;
    for (int q = G.first; q < G.first + G.count; ++q) n += (nrev < 0 || Lo.order[q] < nrev) ? 1 : 0;
    for (int q = G.first; q < G.first + n; ++q)
      if (!(nrev < 0 || Lo.order[q] < nrev)) return SHOT_E_UNSUPPORTED;
    rev_count[gi] = n;
  }
  if (nrev >= 0 && !fwd_info) return SHOT_E_UNSUPPORTED;  // forward-only items need the one-pass form
  bool reverse_phase = false;
  auto each = [&](auto&& fn) -> shot_status {
    for (size_t gi = 0; gi < Lo.groups.size(); ++gi) {
      Group G = Lo.groups[gi];
      if (reverse_phase) {
        G.count = rev_count[gi];
        if (G.count == 0) continue;
      }
      shot_status st = fn(G, P->grids[G.grid]);
      if (st != SHOT_OK) return st;
    }
    return SHOT_OK;
  };
  auto leg = [&](const Group& G, const GridRec& g, cpx<T>* spec) {
    LegArgs<T> la = leg_args<T>(g, G, W, Lo.Lmax, Lo);
    la.spec = spec;
    return run_leg<T>(P, g, la, s);
  };
  // ---- forward sweep with checkpoints of (v-hat_k, s_k) at k = CK, 2CK, ...
  // (none when one segment holds every iteration: the sweep is skipped)
  if (nck > 0)
    ST_TRY(each([&](const Group& G, const GridRec& g) {
      RowArgs<T> a = base_args(G, g);
      a.mode = ROW_INIT;
      return run_rows<T>(P, a, G.count, s);
    }));
  for (int k = 1; nck > 0 && k <= Tit; ++k) {
    ST_TRY(each([&](const Group& G, const GridRec& g) {
      shot_status st = leg(G, g, W.spec);
      if (st != SHOT_OK) return st;
      RowArgs<T> a = base_args(G, g);
      a.mode = ROW_SINK_U;
      a.k = k;
      return run_rows<T>(P, a, G.count, s);
    }));
    ST_TRY(each([&](const Group& G, const GridRec& g) {
      shot_status st = leg(G, g, W.spec);
      if (st != SHOT_OK) return st;
      RowArgs<T> a = base_args(G, g);
      a.mode = ROW_SINK_V;
      a.k = k;
      return run_rows<T>(P, a, G.count, s);
    }));
    if (k % CK == 0 && k < Tit) {
      const int c = k / CK - 1;
      HIP_TRY(hipMemcpyAsync(ckv + F * c, W.vbuf[k & 1], sizeof(T) * F, hipMemcpyDeviceToDevice, s));
      for (const Group& G : Lo.groups) {
        RowArgs<T> a = base_args(G, P->grids[G.grid]);
        HIP_TRY(launch_gauge<T>(a, G.count, k, ckg + (size_t)c * nitems, s));
      }
    }
  }
  // ---- reverse sweep, one segment at a time
  bool started = false;
  for (int seg = nck; seg >= 0; --seg) {
    const int k0 = seg * CK;                 // state after iteration k0 is the checkpoint
    const int k1 = std::min(k0 + CK, Tit);
    // recompute iterations k0+1..k1, keeping u-hat, v-hat and s of each
    ST_TRY(each([&](const Group& G, const GridRec& g) {
      RowArgs<T> a = base_args(G, g);
      if (k0 == 0) {
        a.mode = ROW_INIT;
      } else {
        a.mode = ROW_FWD;
        a.in = ckv + F * (size_t)(seg - 1);
        a.wts_in = 1;
      }
      return run_rows<T>(P, a, G.count, s);
    }));
    for (int k = k0 + 1; k <= k1; ++k) {
      const int slot = k - k0 - 1;
      ST_TRY(each([&](const Group& G, const GridRec& g) {
        shot_status st = leg(G, g, W.spec);
        if (st != SHOT_OK) return st;
        RowArgs<T> a = base_args(G, g);
        a.mode = ROW_SINK_U;
        a.k = k;
        a.ubuf0 = a.ubuf1 = hu + F * slot;
        if (k == k0 + 1 && k0 > 0) a.gk = ckg + (size_t)(seg - 1) * nitems;
        if (fwd_info && k - 1 >= 1 && (k - 1) % C == 0) a.chk_slot = (k - 1) / C - 1;
        return run_rows<T>(P, a, G.count, s);
      }));
      if (!unbal)  // s_k = sum u-hat_k
        for (const Group& G : Lo.groups) {
          RowArgs<T> a = base_args(G, P->grids[G.grid]);
          HIP_TRY(launch_gauge<T>(a, G.count, k, gh + (size_t)slot * nitems, s));
        }
      ST_TRY(each([&](const Group& G, const GridRec& g) {
        shot_status st = leg(G, g, W.spec);
        if (st != SHOT_OK) return st;
        RowArgs<T> a = base_args(G, g);
        a.mode = ROW_SINK_V;
        a.k = k;
        a.vbuf0 = a.vbuf1 = hv + F * slot;
        return run_rows<T>(P, a, G.count, s);
      }));
      if (unbal)  // (g_k, S_A, S_B): needs both halves' partial sums
        for (const Group& G : Lo.groups) {
          RowArgs<T> a = base_args(G, P->grids[G.grid]);
          HIP_TRY(launch_gauge3<T>(a, G.count, k, gh + (size_t)slot * nitems * 3, s));
        }
    }
    if (fwd_info) {
      // the forward pass is complete (one segment): e_marg of the returned
      // scalings, potentials' cost and the reports, as at the end of solve_impl
      const int final_slot = (Tit % C == 0) ? Tit / C - 1 : nslot - 1;
      T* u_last = hu + F * (size_t)(Tit - 1);
      T* v_last = hv + F * (size_t)(Tit - 1);
      ST_TRY(each([&](const Group& G, const GridRec& g) {
        shot_status st = leg(G, g, W.spec);
        if (st != SHOT_OK) return st;
        RowArgs<T> a = base_args(G, g);
        a.mode = ROW_CHECK;
        a.k = Tit + 1;
        a.chk_slot = final_slot;
        a.ubuf0 = a.ubuf1 = u_last;
        a.vbuf0 = a.vbuf1 = v_last;
        return run_rows<T>(P, a, G.count, s);
      }));
      ST_TRY(finish_solve<T>(P, Lo, W, nitems, Tit, C, final_slot, 0.0, nullptr, nullptr, fwd_info, fwd_mass, s,
                             u_last, v_last));
    }
    // walk the segment backwards
    reverse_phase = true;
    if (unbal) {
      for (int k = k1; k > k0; --k) {
        const int slot = k - k0 - 1;
        auto hist = [&](RowArgs<T>& a) {
          a.k = k;
          a.spec = specA;
          a.ubuf0 = a.ubuf1 = hu + F * slot;
          a.vbuf0 = a.vbuf1 = hv + F * slot;
          a.gk = gh + (size_t)slot * nitems * 3;
        };
        // v-bar_k: from the cost at k = T, else K^T of the A-bar_{k+1} spectrum heat-applied below
        ST_TRY(each([&](const Group& G, const GridRec& g) {
          RowArgs<T> a = base_args(G, g);
          a.mode = ROW_ADJU_V1;
          hist(a);
          return run_rows<T>(P, a, G.count, s);
        }));
        ST_TRY(each([&](const Group& G, const GridRec& g) {
          RowArgs<T> a = base_args(G, g);
          a.mode = ROW_ADJU_B;
          hist(a);
          return run_rows<T>(P, a, G.count, s);
        }));
        ST_TRY(each([&](const Group& G, const GridRec& g) {
          shot_status st = leg(G, g, specA);
          if (st != SHOT_OK) return st;
          RowArgs<T> a = base_args(G, g);
          a.mode = ROW_ADJU_A;
          hist(a);
          return run_rows<T>(P, a, G.count, s);
        }));
        if (k == 1) break;
        ST_TRY(each([&](const Group& G, const GridRec& g) { return leg(G, g, specA); }));
      }
      continue;
    }
    for (int k = k1; k > k0; --k) {
      const int slot = k - k0 - 1;
      if (!started) {
        ST_TRY(each([&](const Group& G, const GridRec& g) {
          RowArgs<T> a = base_args(G, g);
          a.mode = ROW_ADJ_START;
          a.k = k;
          a.spec = specA;
          a.ubuf0 = a.ubuf1 = hu + F * slot;
          a.vbuf0 = a.vbuf1 = hv + F * slot;
          a.gk = gh + (size_t)slot * nitems;
          return run_rows<T>(P, a, G.count, s);
        }));
        started = true;
      }
      ST_TRY(each([&](const Group& G, const GridRec& g) {
        shot_status st = leg(G, g, specA);
        if (st != SHOT_OK) return st;
        RowArgs<T> a = base_args(G, g);
        a.mode = ROW_ADJ_A;
        a.k = k;
        a.spec = specA;
        a.ubuf0 = a.ubuf1 = hu + F * slot;
        a.gk = gh + (size_t)slot * nitems;
        return run_rows<T>(P, a, G.count, s);
      }));
      if (k == 1) break;
      ST_TRY(each([&](const Group& G, const GridRec& g) {
        shot_status st = leg(G, g, specA);
        if (st != SHOT_OK) return st;
        RowArgs<T> a = base_args(G, g);
        a.mode = ROW_ADJ_VB;
        a.k = k;
        a.spec = specA;
        if (k - 1 > k0) {
          a.vbuf0 = a.vbuf1 = hv + F * (slot - 1);
          a.gk = gh + (size_t)(slot - 1) * nitems;
        } else {  // iteration k0: the checkpoint
          a.vbuf0 = a.vbuf1 = ckv + F * (size_t)(seg - 1);
          a.gk = ckg + (size_t)(seg - 1) * nitems;
        }
        return run_rows<T>(P, a, G.count, s);
      }));
    }
  }
  *pbar_out = gA;
  *qbar_out = gB;
  return SHOT_OK;
}

// Combine per-item fields into per-pair gradients on the device.
template <typename T>
shot_status combine_pairs(shot_plan_s* P, const std::vector<CombineDev>& dv, T* out, hipStream_t s) {
  if (dv.empty()) return SHOT_OK;
  long long maxn = 0;
  for (const auto& d : dv) maxn = std::max(maxn, d.n);
  void* dd = nullptr;
  HIP_TRY(hipMalloc(&dd, sizeof(CombineDev) * dv.size()));
  hipError_t e = hipMemcpyAsync(dd, dv.data(), sizeof(CombineDev) * dv.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_combine<T>(static_cast<CombineDev*>(dd), (int)dv.size(), maxn, out, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dd);
  if (e != hipSuccess) return hip_fail(e, "gradient combine", __LINE__);
  (void)P;
  return SHOT_OK;
}

template <typename T>
shot_status divergence_grad_impl(shot_plan_s* P, const int32_t* gop, int npairs, const shot_params* params,
                                 const void* p, const void* q, double* S_out, T* dS, int mode, int CK,
                                 shot_solve_info* info, hipStream_t s) {
  Layout Lp;
  ST_TRY(make_layout(P, gop, npairs, Lp));
  // unrolled: balanced or unbalanced, every pair of a call the same; the
  // envelope form (the potentials' formula of Sec. 4.2.2) is balanced only
  const bool unbal = !std::isinf(params[0].tau);
  for (int i = 0; i < npairs; ++i) {
    ST_TRY(check_params(params[i]));
    if (params[i].tol != 0 || std::isinf(params[i].tau) == unbal || (mode == 1 && unbal)) return SHOT_E_UNSUPPORTED;
  }
  const T* pb = static_cast<const T*>(p);
  const T* qb = static_cast<const T*>(q);
  if (mode == 0 && CK <= 0) {
    // one forward pass over all three solves of every pair keeps the whole
    // history and reports them; the reverse sweep then runs the (p,q) and (p,p)
    // solves, which come first (the (q,q) solves follow, forward only)
    SolveSpec S2;
    for (int i = 0; i < npairs; ++i) {
      const T* pi = pb + Lp.user_foff[i];
      const T* qi = qb + Lp.user_foff[i];
      const void* ps[2] = {pi, pi};
      const void* qs[2] = {qi, pi};
      for (int r = 0; r < 2; ++r) {
        S2.grid.push_back(gop[i]);
        S2.prm.push_back(params[i]);
        S2.p.push_back(ps[r]);
        S2.q.push_back(qs[r]);
      }
    }
    for (int i = 0; i < npairs; ++i) {
      const T* qi = qb + Lp.user_foff[i];
      S2.grid.push_back(gop[i]);
      S2.prm.push_back(params[i]);
      S2.p.push_back(qi);
      S2.q.push_back(qi);
    }
    Layout L2;
    ST_TRY(make_layout(P, S2.grid.data(), 3 * npairs, L2));
    if (whole_history_fits<T>(L2.field_total, params[0].max_iter)) {
      std::vector<shot_solve_info> inf2(3 * (size_t)npairs), inf(3 * (size_t)npairs);
      std::vector<double> mass2(6 * (size_t)npairs), mass(6 * (size_t)npairs);
      T* gA = nullptr;
      T* gB = nullptr;
      ST_TRY(adjoint_impl<T>(P, S2, 0, &gA, &gB, L2, s, inf2.data(), mass2.data(), 2 * npairs));
      for (int i = 0; i < npairs; ++i) {
        for (int r = 0; r < 3; ++r) {
          const int u = r < 2 ? 2 * i + r : 2 * npairs + i;
          inf[3 * i + r] = inf2[u];
          mass[6 * i + 2 * r] = mass2[2 * u];
          mass[6 * i + 2 * r + 1] = mass2[2 * u + 1];
        }
      }
      combine_divergence(params, npairs, inf.data(), mass.data(), S_out);
      if (info) std::copy(inf.begin(), inf.end(), info);
      std::vector<CombineDev> dv(npairs);
      for (int i = 0; i < npairs; ++i) {
        const GridRec& g = P->grids[gop[i]];
        CombineDev& d = dv[i];
        d.off_out = Lp.user_foff[i];
        d.off1 = L2.user_foff[2 * i];      // p-bar of (p,q)
        d.off2 = L2.user_foff[2 * i + 1];  // p-bar of (p,p)
        d.off3 = L2.user_foff[2 * i + 1];  // q-bar of (p,p)
        d.x1 = gA;
        d.x2 = gA;
        d.x3 = gB;
        d.mul_area = 0;
        d.coef = params[i].eps * (mass[6 * i] - mass[6 * i + 1]);
        d.nlat = g.d.nlat;
        d.nlon = g.d.nlon;
        d.n = g.n();
        d.equal_area = g.hp ? 1 : 0;
        d.h = g.h;
        d.aw = g.d_aw;
      }
      return combine_pairs<T>(P, dv, dS, s);
    }
  }
  // forward divergence: three solves per pair (potentials kept for the envelope form)
  SolveSpec S3;
  for (int i = 0; i < npairs; ++i) {
    const T* pi = pb + Lp.user_foff[i];
    const T* qi = qb + Lp.user_foff[i];
    const void* ps[3] = {pi, pi, qi};
    const void* qs[3] = {qi, pi, qi};
    for (int r = 0; r < 3; ++r) {
      S3.grid.push_back(gop[i]);
      S3.prm.push_back(params[i]);
      S3.p.push_back(ps[r]);
      S3.q.push_back(qs[r]);
    }
  }
  std::vector<shot_solve_info> inf(3 * (size_t)npairs);
  std::vector<double> mass(6 * (size_t)npairs);
  Layout L3;
  ST_TRY(make_layout(P, S3.grid.data(), 3 * npairs, L3));
  T* phi3 = nullptr;
  T* psi3 = nullptr;
  if (mode == 1) {
    const size_t F3 = (size_t)L3.field_total;
    ST_TRY(grow(P->ws2, 2 * F3 * sizeof(T)));
    phi3 = static_cast<T*>(P->ws2.p);
    psi3 = phi3 + F3;
  }
  ST_TRY(solve_impl<T>(P, S3, phi3, psi3, inf.data(), mass.data(), s));
  combine_divergence(params, npairs, inf.data(), mass.data(), S_out);
  if (info) std::copy(inf.begin(), inf.end(), info);
  std::vector<CombineDev> dv(npairs);
  if (mode == 1) {
    for (int i = 0; i < npairs; ++i) {
      const GridRec& g = P->grids[gop[i]];
      CombineDev& d = dv[i];
      d.off_out = Lp.user_foff[i];
      d.off1 = L3.user_foff[3 * i];      // phi_pq
      d.off2 = L3.user_foff[3 * i + 1];  // phi_pp
      d.off3 = L3.user_foff[3 * i + 1];  // psi_pp
      d.x1 = phi3;
      d.x2 = phi3;
      d.x3 = psi3;
      d.mul_area = 1;
      d.coef = params[i].eps * (mass[6 * i] - mass[6 * i + 1]);
      d.nlat = g.d.nlat;
      d.nlon = g.d.nlon;
      d.n = g.n();
      d.equal_area = g.hp ? 1 : 0;
      d.h = g.h;
      d.aw = g.d_aw;
    }
    return combine_pairs<T>(P, dv, dS, s);
  }
  // unrolled: reverse sweeps of the (p,q) and (p,p) solves
  SolveSpec S2;
  for (int i = 0; i < npairs; ++i)
    for (int r = 0; r < 2; ++r) {
      S2.grid.push_back(gop[i]);
      S2.prm.push_back(params[i]);
      S2.p.push_back(S3.p[3 * i + r]);
      S2.q.push_back(S3.q[3 * i + r]);
    }
  Layout L2;
  T* gA = nullptr;
  T* gB = nullptr;
  ST_TRY(adjoint_impl<T>(P, S2, CK, &gA, &gB, L2, s));
  for (int i = 0; i < npairs; ++i) {
    const GridRec& g = P->grids[gop[i]];
    CombineDev& d = dv[i];
    d.off_out = Lp.user_foff[i];
    d.off1 = L2.user_foff[2 * i];      // p-bar of (p,q)
    d.off2 = L2.user_foff[2 * i + 1];  // p-bar of (p,p)
    d.off3 = L2.user_foff[2 * i + 1];  // q-bar of (p,p)
    d.x1 = gA;
    d.x2 = gA;
    d.x3 = gB;
    d.mul_area = 0;
    d.coef = params[i].eps * (mass[6 * i] - mass[6 * i + 1]);
    d.nlat = g.d.nlat;
    d.nlon = g.d.nlon;
    d.n = g.n();
    d.equal_area = g.hp ? 1 : 0;
    d.h = g.h;
    d.aw = g.d_aw;
  }
  return combine_pairs<T>(P, dv, dS, s);
}

template <typename T>
shot_status regional_rms_impl(shot_plan_s* P, const int32_t* gop, int npairs, const void* d, const double* bands,
                              int nbands, double* out, hipStream_t s) {
  Layout Lo;
  ST_TRY(make_layout(P, gop, npairs, Lo));
  Work<T> W;
  ST_TRY(carve<T>(P, Lo, npairs, false, 0, W));
  std::fill(out, out + (size_t)npairs * nbands, std::nan(""));
  for (const Group& G : Lo.groups) {
    const GridRec& g = P->grids[G.grid];
    const int nlat = g.d.nlat;
    std::vector<long long> foff(G.count);
    for (int i = 0; i < G.count; ++i) foff[i] = Lo.user_foff[Lo.order[G.first + i]];
    long long* d_foff = nullptr;
    double* d_aw = nullptr;
    double* d_out = nullptr;
    ST_TRY(upload((void**)&d_foff, foff, s));
    shot_status sa = upload((void**)&d_aw, g.aw_host, s);
    if (sa != SHOT_OK) { (void)hipFree(d_foff); return sa; }
    hipError_t e = hipMalloc((void**)&d_out, sizeof(double) * 3 * nlat * G.count);
    if (e != hipSuccess) {
      (void)hipFree(d_foff);
      (void)hipFree(d_aw);
      return hip_fail(e, "hipMalloc", __LINE__);
    }
    RowArgs<T> a = row_args<T>(P, g, Lo, G, W, npairs);
    e = launch_row_stats<T>(a, G.count, static_cast<const T*>(d), d_foff, d_aw, d_out, s);
    std::vector<double> st((size_t)3 * nlat * G.count);
    if (e == hipSuccess) e = hipMemcpyAsync(st.data(), d_out, sizeof(double) * st.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_foff);
    (void)hipFree(d_aw);
    (void)hipFree(d_out);
    if (e != hipSuccess) return hip_fail(e, "regional statistics", __LINE__);
    for (int i = 0; i < G.count; ++i) {
      const int ui = Lo.order[G.first + i];
      const double* r = st.data() + (size_t)i * nlat * 3;
      double A0 = 0, A1 = 0;
      for (int j = 0; j < nlat; ++j) { A0 += r[3 * j]; A1 += r[3 * j + 1]; }
      const double mean = A1 / A0;
      for (int b = 0; b < nbands; ++b) {
        double B0 = 0, B1 = 0, B2 = 0;
        for (int j = 0; j < nlat; ++j) {
          const double lat = std::asin(std::max(-1.0, std::min(1.0, g.x[j]))) * 180.0 / M_PI;
          // rows within 1e-9 degree of a bound lie on it (equiangular rows hit bounds exactly)
          if (lat > bands[2 * b] + 1e-9 && lat < bands[2 * b + 1] - 1e-9) {
            B0 += r[3 * j];
            B1 += r[3 * j + 1];
            B2 += r[3 * j + 2];
          }
        }
        if (B0 > 0) out[(size_t)ui * nbands + b] = std::sqrt(std::max(0.0, (B2 - 2 * mean * B1 + mean * mean * B0) / B0));
      }
    }
  }
  return SHOT_OK;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* shot_last_error(void) { return g_last_error; }

const char* shot_status_string(int32_t s) {
  switch (s) {
    case SHOT_OK: return "ok";
    case SHOT_E_INVALID: return "invalid argument";
    case SHOT_E_NOMEM: return "out of device memory";
    case SHOT_E_HIP: return "HIP runtime error";
    case SHOT_E_UNSUPPORTED: return "unsupported configuration";
    case SHOT_W_NOT_CONVERGED: return "not converged (e_marg >= tol)";
    case SHOT_E_BREAKDOWN: return "breakdown: heat-kernel output <= 0 or non-finite";
    default: return "unknown status";
  }
}

shot_status shot_sht_plan(shot_plan_t* out, const shot_grid_desc* grids, int32_t ngrids,
                          int32_t precision, int32_t legendre_mode, void* stream) {
  if (!out) return SHOT_E_INVALID;
  *out = nullptr;
  if (!grids || ngrids <= 0) return SHOT_E_INVALID;
  if (precision < SHOT_FP64 || precision > SHOT_BF16X3_MFMA) return SHOT_E_INVALID;
  // split bfloat16 operands are formed from the recurrence's values; no table form
  if (precision == SHOT_BF16X3_MFMA && legendre_mode == SHOT_LEG_TABLE) return SHOT_E_UNSUPPORTED;
  if (legendre_mode < SHOT_LEG_AUTO || legendre_mode > SHOT_LEG_RECURRENCE) return SHOT_E_INVALID;
  for (int i = 0; i < ngrids; ++i) {
    const shot_grid_desc& d = grids[i];
    if (d.kind != SHOT_GRID_GAUSS_LEGENDRE && d.kind != SHOT_GRID_CLENSHAW_CURTIS && d.kind != SHOT_GRID_HEALPIX &&
        d.kind != SHOT_GRID_LOBATTO)
      return SHOT_E_INVALID;
    if (d.kind == SHOT_GRID_HEALPIX) {
      if (d.L < 1 || d.nlon < 4 || d.nlon % 4 != 0 || d.nlat != d.nlon - 1) return SHOT_E_INVALID;
      if (d.nlon > 2048) return SHOT_E_UNSUPPORTED;
    } else {
      if (d.nlat < 2 || d.nlon < 2 || d.L < 1 || d.nlon < 2 * d.L - 1) return SHOT_E_INVALID;
      // any row length: radices 4, 2, 3, 5 and a direct stage per larger prime
      if (d.nlon > 2048 || fft_factors(d.nlon).size() > 8) return SHOT_E_UNSUPPORTED;
    }
    // one order's inputs and coefficients must fit the Legendre kernel's LDS
    const size_t cs = precision == SHOT_FP64 ? 16 : 8;
    if ((size_t)(2 * ((d.nlat + 1) / 2) + d.L) * cs > 60 * 1024) return SHOT_E_UNSUPPORTED;
    if (legendre_mode == SHOT_LEG_RECURRENCE &&
        ((d.nlat + 1) / 2 > 1024 || (size_t)(d.L + 15) / 16 * 16 * 32 > 56 * 1024))
      return SHOT_E_UNSUPPORTED;
  }
  shot_plan_s* P = new (std::nothrow) shot_plan_s();
  if (!P) return SHOT_E_NOMEM;
  P->prec = precision;
  {
    hipError_t e = hipGetDevice(&P->dev);
    if (e != hipSuccess) { delete P; return hip_fail(e, "hipGetDevice", __LINE__); }
  }
  {
    shot_status st = scratch_setup(P->dev);  // the device is current here
    if (st != SHOT_OK) { delete P; return st; }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  P->grids.resize(ngrids);
  for (int i = 0; i < ngrids; ++i) {
    P->grids[i].d = grids[i];
    shot_status st = build_grid(P, P->grids[i], legendre_mode, s);
    if (st != SHOT_OK) {
      shot_plan_destroy(P);
      return st;
    }
  }
  *out = P;
  return SHOT_OK;
}

shot_status shot_plan_destroy(shot_plan_t P) {
  if (!P) return SHOT_OK;
  (void)hipDeviceSynchronize();
  for (auto& g : P->grids) free_grid(g);
  drop_graph(P);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  for (auto b : P->branch) (void)hipStreamDestroy(b);
  for (auto e : P->bev) (void)hipEventDestroy(e);
  if (P->ws.p) (void)hipFree(P->ws.p);
  if (P->ws2.p) (void)hipFree(P->ws2.p);
  for (auto e : P->evpool) (void)hipEventDestroy(e);
  delete P;
  return SHOT_OK;
}

shot_status shot_plan_grid(shot_plan_t P, int32_t grid, double* x_out, double* w_out) {
  if (!P || grid < 0 || grid >= (int)P->grids.size()) return SHOT_E_INVALID;
  const GridRec& g = P->grids[grid];
  if (x_out) std::copy(g.x.begin(), g.x.end(), x_out);
  if (w_out) std::copy(g.w.begin(), g.w.end(), w_out);
  return SHOT_OK;
}

shot_status shot_plan_area_weights(shot_plan_t P, int32_t grid, double* a_out) {
  if (!P || grid < 0 || grid >= (int)P->grids.size() || !a_out) return SHOT_E_INVALID;
  const GridRec& g = P->grids[grid];
  if (g.hp) {
    // every pixel of a HEALPix grid has the area 4 pi / Npix
    std::fill(a_out, a_out + g.n(), 4.0 * M_PI / (double)g.n());
    return SHOT_OK;
  }
  // latitude-longitude grids: a_{jk} = w_j * 2 pi / nlon, row-major
  const int nlat = g.d.nlat, nlon = g.d.nlon;
  for (int j = 0; j < nlat; ++j) std::fill(a_out + (size_t)j * nlon, a_out + (size_t)(j + 1) * nlon, g.w[j] * 2.0 * M_PI / nlon);
  return SHOT_OK;
}

const char* shot_build_id(void) { return SHOT_SOURCE_HASH; }

shot_status shot_gradient_regional_rms(shot_plan_t P, const int32_t* goi, int32_t npairs, const void* d,
                                       const double* bands, int32_t nbands, double* out, void* stream) {
  if (!P || !goi || npairs <= 0 || !ptr_ok(d) || !bands || nbands <= 0 || !out) return SHOT_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  return P->prec == SHOT_FP64 ? regional_rms_impl<double>(P, goi, npairs, d, bands, nbands, out, s)
                              : regional_rms_impl<float>(P, goi, npairs, d, bands, nbands, out, s);
}

shot_status shot_plan_ring(shot_plan_t P, int32_t grid, int32_t* npix_out, double* phi0_out) {
  if (!P || grid < 0 || grid >= (int)P->grids.size()) return SHOT_E_INVALID;
  const GridRec& g = P->grids[grid];
  for (int r = 0; r < g.d.nlat; ++r) {
    if (npix_out) npix_out[r] = g.hp ? g.ring_npix[r] : g.d.nlon;
    if (phi0_out) phi0_out[r] = g.hp ? g.ring_phi0[r] : 0.0;
  }
  return SHOT_OK;
}

shot_status shot_sht_analysis(shot_plan_t P, const int32_t* goi, int32_t nitems, const void* f,
                              void* coeffs, void* stream) {
  if (!P || !ptr_ok(f) || !ptr_ok(coeffs)) return SHOT_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  return P->prec == SHOT_FP64 ? sht_impl<double>(P, goi, nitems, f, coeffs, true, s)
                              : sht_impl<float>(P, goi, nitems, f, coeffs, true, s);
}

shot_status shot_sht_synthesis(shot_plan_t P, const int32_t* goi, int32_t nitems, const void* coeffs,
                               void* f, void* stream) {
  if (!P || !ptr_ok(f) || !ptr_ok(coeffs)) return SHOT_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  return P->prec == SHOT_FP64 ? sht_impl<double>(P, goi, nitems, coeffs, f, false, s)
                              : sht_impl<float>(P, goi, nitems, coeffs, f, false, s);
}

shot_status shot_heat_apply(shot_plan_t P, const int32_t* goi, int32_t nitems, const double* t,
                            const void* v, void* out, int32_t transpose, void* stream) {
  if (!P || !t || !ptr_ok(v) || !ptr_ok(out) || v == out) return SHOT_E_INVALID;
  for (int i = 0; i < nitems; ++i)
    if (!(t[i] >= 0) || !std::isfinite(t[i])) return SHOT_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  return P->prec == SHOT_FP64 ? heat_apply_impl<double>(P, goi, nitems, t, v, out, transpose, s)
                              : heat_apply_impl<float>(P, goi, nitems, t, v, out, transpose, s);
}

shot_status shot_heat_apply_noalloc(shot_plan_t P, const int32_t* goi, int32_t nitems, const double* t,
                                    const void* v, void* out, int32_t transpose, void* stream) {
  if (!P || !t || !ptr_ok(v) || !ptr_ok(out) || v == out) return SHOT_E_INVALID;
  for (int i = 0; i < nitems; ++i)
    if (!(t[i] >= 0) || !std::isfinite(t[i])) return SHOT_E_INVALID;
  char* base = scratch_of(P->dev);
  if (!base) return SHOT_E_INVALID;  // no plan was ever made on this device
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  return P->prec == SHOT_FP64
             ? heat_apply_impl<double>(P, goi, nitems, t, v, out, transpose, s, base, SHOT_NOALLOC_SCRATCH_BYTES)
             : heat_apply_impl<float>(P, goi, nitems, t, v, out, transpose, s, base, SHOT_NOALLOC_SCRATCH_BYTES);
}

shot_status shot_sinkhorn_solve(shot_plan_t P, const int32_t* goi, int32_t nitems,
                                const shot_params* params, const void* p, const void* q, void* phi,
                                void* psi, shot_solve_info* info, void* stream) {
  if (!P || !goi || nitems <= 0 || !params || !ptr_ok(p) || !ptr_ok(q) || !info) return SHOT_E_INVALID;
  Layout Lo;
  shot_status st = make_layout(P, goi, nitems, Lo);
  if (st != SHOT_OK) return st;
  SolveSpec S;
  S.grid.assign(goi, goi + nitems);
  S.prm.assign(params, params + nitems);
  const size_t es = field_elem(P);
  for (int i = 0; i < nitems; ++i) {
    S.p.push_back(static_cast<const char*>(p) + Lo.user_foff[i] * es);
    S.q.push_back(static_cast<const char*>(q) + Lo.user_foff[i] * es);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  st = P->prec == SHOT_FP64
           ? solve_impl<double>(P, S, static_cast<double*>(phi), static_cast<double*>(psi), info, nullptr, s)
           : solve_impl<float>(P, S, static_cast<float*>(phi), static_cast<float*>(psi), info, nullptr, s);
  if (st != SHOT_OK) return st;
  return worst(info, nitems);
}

shot_status shot_sinkhorn_divergence(shot_plan_t P, const int32_t* gop, int32_t npairs,
                                     const shot_params* params, const void* p, const void* q,
                                     double* S_out, shot_solve_info* info, void* stream) {
  if (!P || !gop || npairs <= 0 || !params || !ptr_ok(p) || !ptr_ok(q) || !S_out) return SHOT_E_INVALID;
  Layout Lo;
  shot_status st = make_layout(P, gop, npairs, Lo);
  if (st != SHOT_OK) return st;
  SolveSpec S;
  const size_t es = field_elem(P);
  for (int i = 0; i < npairs; ++i) {
    const void* pi = static_cast<const char*>(p) + Lo.user_foff[i] * es;
    const void* qi = static_cast<const char*>(q) + Lo.user_foff[i] * es;
    const void* ps[3] = {pi, pi, qi};
    const void* qs[3] = {qi, pi, qi};
    for (int r = 0; r < 3; ++r) {
      S.grid.push_back(gop[i]);
      S.prm.push_back(params[i]);
      S.p.push_back(ps[r]);
      S.q.push_back(qs[r]);
    }
  }
  std::vector<shot_solve_info> inf(3 * (size_t)npairs);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  std::vector<double> mass(6 * (size_t)npairs);
  st = P->prec == SHOT_FP64 ? solve_impl<double>(P, S, nullptr, nullptr, inf.data(), mass.data(), s)
                            : solve_impl<float>(P, S, nullptr, nullptr, inf.data(), mass.data(), s);
  if (st != SHOT_OK) return st;
  combine_divergence(params, npairs, inf.data(), mass.data(), S_out);
  if (info) std::copy(inf.begin(), inf.end(), info);
  return worst(inf.data(), 3 * npairs);
}

shot_status shot_sinkhorn_divergence_grad(shot_plan_t P, const int32_t* gop, int32_t npairs,
                                          const shot_params* params, const void* p, const void* q,
                                          double* S_out, void* dS_dp, int32_t mode,
                                          int32_t checkpoint_every, shot_solve_info* info,
                                          void* stream) {
  if (!P || !gop || npairs <= 0 || !params || !ptr_ok(p) || !ptr_ok(q) || !S_out || !ptr_ok(dS_dp))
    return SHOT_E_INVALID;
  if (mode != 0 && mode != 1) return SHOT_E_INVALID;
  if (checkpoint_every < 0) return SHOT_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(P->dev));
  std::vector<shot_solve_info> inf(3 * (size_t)npairs);
  shot_status st =
      P->prec == SHOT_FP64
          ? divergence_grad_impl<double>(P, gop, npairs, params, p, q, S_out, static_cast<double*>(dS_dp),
                                         mode, checkpoint_every, inf.data(), s)
          : divergence_grad_impl<float>(P, gop, npairs, params, p, q, S_out, static_cast<float*>(dS_dp),
                                        mode, checkpoint_every, inf.data(), s);
  if (st != SHOT_OK) return st;
  if (info) std::copy(inf.begin(), inf.end(), info);
  return worst(inf.data(), 3 * npairs);
}

shot_status shot_plan_set_tuning(shot_plan_t P, int32_t grid, int32_t items_per_block,
                                 int32_t chains_per_thread) {
  if (!P || grid < 0 || grid >= (int)P->grids.size()) return SHOT_E_INVALID;
  GridRec& g = P->grids[grid];
  if (items_per_block != 0 && items_per_block != 1 && items_per_block != 2 && items_per_block != 4 &&
      items_per_block != 8 && !(items_per_block == 16 && g.tab_kind == TAB_RECUR))
    return SHOT_E_INVALID;
  if (g.tab_kind == TAB_RECUR) {
    if (chains_per_thread != 0 && !recur_jpt_valid(g.h, chains_per_thread)) return SHOT_E_INVALID;
  } else if (chains_per_thread != 0) {
    const bool mma = mma_table(g);
    if (!(chains_per_thread == -1 || (mma && (chains_per_thread == 1 || chains_per_thread == 2 ||
                                                chains_per_thread == 4))))
      return SHOT_E_INVALID;
  }
  g.tune_ib = items_per_block;
  g.tune_jpt = chains_per_thread;
  return SHOT_OK;
}

shot_status shot_plan_get_tuning(shot_plan_t P, int32_t grid, int32_t* items_per_block,
                                 int32_t* chains_per_thread) {
  if (!P || grid < 0 || grid >= (int)P->grids.size()) return SHOT_E_INVALID;
  const GridRec& g = P->grids[grid];
  if (items_per_block) *items_per_block = g.tune_ib;
  if (chains_per_thread) *chains_per_thread = g.tune_jpt;
  return SHOT_OK;
}

shot_status shot_autotune(shot_plan_t P, int32_t grid, int32_t nitems, void* stream) {
  if (!P || grid < 0 || grid >= (int)P->grids.size() || nitems <= 0) return SHOT_E_INVALID;
  HIP_TRY(hipSetDevice(P->dev));
  hipStream_t s = static_cast<hipStream_t>(stream);
  GridRec& g = P->grids[grid];
  std::vector<int32_t> goi(nitems, grid);
  Layout Lo;
  ST_TRY(make_layout(P, goi.data(), nitems, Lo));
  const bool f64 = P->prec == SHOT_FP64;
  shot_status st = f64 ? autotune_impl<double>(P, g, Lo, nitems, s) : autotune_impl<float>(P, g, Lo, nitems, s);
  return st;
}

shot_status shot_plan_set_graphs(shot_plan_t P, int32_t enable) {
  if (!P) return SHOT_E_INVALID;
  P->graphs = enable != 0;
  if (!P->graphs) drop_graph(P);
  return SHOT_OK;
}

shot_status shot_profile_enable(shot_plan_t P, int32_t enable) {
  if (!P) return SHOT_E_INVALID;
  drop_graph(P);  // captured graphs hold the previous event records
  if (enable) {
    P->timed.clear();
    P->evnext = 0;
  }
  P->prof = enable != 0;
  return SHOT_OK;
}

shot_status shot_profile_read(shot_plan_t P, int32_t cls, int64_t* launches, double* total_ms) {
  if (!P || !launches || !total_ms) return SHOT_E_INVALID;
  int64_t n = 0;
  double ms = 0.0;
  for (const Timed& t : P->timed) {
    if (t.cls != cls) continue;
    HIP_TRY(hipEventSynchronize(t.b));
    float e = 0.f;
    HIP_TRY(hipEventElapsedTime(&e, t.a, t.b));
    ms += e;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  return SHOT_OK;
}

}  // extern "C"
