// Internal types shared by the libshot host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "host_math.h"

namespace shot {

template <typename T>
struct cpx {
  T x, y;
};

// Per-item descriptor, resident on the device for the duration of a call.
struct ItemDev {
  long long foff;      // element offset of the item's fields (p, q, phi, psi, in, out, u, v)
  long long soff;      // complex-element offset of the item's spectral workspace
  long long coff;      // complex-element offset of the item's packed (m, l) coefficients
  const void* p;       // this item's first marginal (device)
  const void* q;       // this item's second marginal (device)
  double eps;          // entropic parameter
  double tau;          // marginal penalty (ignored when balanced)
  double lam;          // tau/(tau+eps): exponent of the unbalanced update
  double eot;          // eps/tau
  int balanced;        // 1: tau = +inf
  int pad;
};

constexpr int RED_SLOTS = 8;

// One mirror pair of rings of a HEALPix grid (ring j and ring nlat-1-j have
// the same length and first-pixel longitude).
constexpr int RING_MAXFAC = 12;
struct RingDev {
  int len;                 // pixels per ring
  int off1, off2;          // first pixel of the northern / southern ring in a field
  int twoff;               // offset of this length's twiddles exp(-2 pi i k/len) in ring_tw
  int nfac;                // factors of len (4, 2, 3, 5, then other primes)
  int fac[RING_MAXFAC];
  // Bluestein transform for lengths with a large prime factor (bm > 0): the
  // length-len DFT as a cyclic convolution of power-of-two length bm
  int bm;                  // convolution length (0: direct stages)
  int bm_nfac;             // factors of bm (4s and a 2)
  int bm_fac[RING_MAXFAC];
  int bm_twoff;            // offset of exp(-2 pi i k/bm), k < bm, in ring_tw
  int ch_off;              // offset of the chirp exp(-i pi n^2/len), n < len, in ring_blu
  int bh_off;              // offset of FFT_bm(filter) / bm in ring_blu
};

// Row kernel modes.
enum RowMode : int {
  ROW_FWD = 0,     // field -> folded spectrum
  ROW_INV = 1,     // folded spectrum -> field
  ROW_SINK_U = 2,  // spectrum of K v -> u-update (+ e_marg residual) -> spectrum of u
  ROW_SINK_V = 3,  // spectrum of K u -> v-update -> spectrum of v
  ROW_CHECK = 4,   // spectrum of K v -> e_marg residual only
  ROW_FINAL = 5,   // potentials and cost partials (no FFT)
  ROW_INIT = 6,    // spectrum of the constant 1 field + norms/masses of p, q
  // adjoint sweep (balanced, see adjoint comments in kernels.hip)
  ROW_ADJ_START = 7,  // final-cost adjoints of u_T, v_T -> B-bar_T; spectrum of B-bar_T
  ROW_ADJ_A = 8,      // K^T B-bar -> u-hat-bar -> A-bar, p-bar; spectrum of A-bar
  ROW_ADJ_VB = 9,     // K^T A-bar = v-bar_{k-1} -> B-bar_{k-1}, q-bar; spectrum of B-bar_{k-1}
  // adjoint sweep of the unbalanced iteration (see kernels.hip): per step k
  ROW_ADJU_V1 = 10,   // v-bar_k (from the cost at k = T, else K^T A-bar_{k+1}) -> vbar, g-bar partials
  ROW_ADJU_B = 11,    // g-bar -> v-hat-bar, q-bar, B-bar_k; spectrum of B-bar_k
  ROW_ADJU_A = 12,    // K^T B-bar -> u-hat-bar, p-bar, A-bar_k; spectrum of A-bar_k
};

template <typename T>
struct RowArgs {
  int nlat, nlon, L, h;
  int hs;             // row-pair stride of the per-item partial-sum arrays (max h over items)
  int nfac;
  int fac[8];
  const cpx<T>* tw;   // nlon forward twiddles exp(-2 pi i k / nlon)
  const T* aw;        // h area weights (rows 0..h-1)
  int item0;          // absolute index of this launch's first item
  const ItemDev* items;
  const int* rpair;   // ring grids: ring pair run by workgroup column b (nullptr: xcd_row_pair order)
  cpx<T>* spec;
  int mode;
  int k;              // iteration number (1-based) for SINK / CHECK / FINAL modes
  int wts_in;         // FWD-like modes: multiply the folded spectrum by a_j
  int wts_out;        // INV: multiply the output rows by a_j
  const T* in;        // FWD: input fields (NULL = constant 1)
  T* out;             // INV: output fields; FINAL: phi
  T* out2;            // FINAL: psi
  T* ubuf0; T* ubuf1; // ping-pong u-hat by iteration parity
  T* vbuf0; T* vbuf1; // ping-pong v-hat by iteration parity
  double* red;        // [2][nitems][hs][RED_SLOTS] per-row-pair partials: 0 u-half sum, 1 v-half sum,
                      // 2/3 u-half min/max of K v, 4/5 v-half min/max of K u
  double* kr;         // [nitems] running min over half-iterations of min(K.)/max(K.)
  int nitems_all;
  double* rhist;      // [nitems][nslot][h] e_marg residual partials
  int nslot;
  int chk_slot;       // slot written by this launch, -1 for none
  int store_field;    // Sinkhorn halves: store the new scaling field (a later
                      // check, the final potentials or the reverse sweep reads
                      // it); 0 skips the store (the next half needs only the
                      // spectrum this launch writes)
  double* prep;       // [nitems][h][4]: sum p^2, sum a p, sum a q, cost partial
  int* brk;           // [nitems] first breakdown iteration (INT_MAX = none)
  // adjoint state (balanced reverse sweep) and gauge overrides
  T* gA;              // p-bar accumulator (layout of fields)
  T* gB;              // q-bar accumulator
  double* adjp;       // [nitems][hs] partial sums of s-bar
  const double* gk;   // [nitems] SINK_U: gauge of iteration k-1 to use instead of the partial sums;
                      // adjoint modes: s of the iteration whose u-hat / v-hat are read
  int kT;             // adjoint: last iteration T (its u-bar term enters ROW_ADJ_A)
  T* vbar;            // unbalanced adjoint: v-bar_k field (layout of fields)
  // spectrum written by a row-split Legendre launch that cut long orders into
  // parts: cut[m] = (parts, first partial slot); nullptr when nothing was cut
  const int2* cut;
  const void* pbuf;   // [chunks][npb][cut_ib][h][2] partial sums (cpx<T>)
  int npb;
  int cut_ib;         // items per Legendre workgroup of that launch
  // HEALPix grids: per row pair ring geometry, twiddles of every ring length,
  // and e^{i m phi0} per (row pair, m < L); nullptr for latitude-longitude grids
  const RingDev* ring;
  const cpx<T>* ring_tw;
  const cpx<T>* ring_ph;
  const cpx<T>* ring_blu;   // HEALPix: Bluestein chirps and filter spectra
  int nbuf;                 // HEALPix: LDS length of each FFT buffer (longest ring or convolution)
};

// Pointwise combination of per-item fields into a per-pair gradient:
// out = wa * (x1 - (x2 + x3)/2) + coef * a, wa = a (potentials) or 1.
struct CombineDev {
  long long off_out, off1, off2, off3;  // element offsets
  long long n;                          // points per field
  double coef;
  int nlat, nlon, h;
  int mul_area;
  int equal_area;                       // every point has area aw[0] (HEALPix)
  const void* aw;   // h area weights (field precision)
  const void* x1; const void* x2; const void* x3;
};

template <typename T>
struct LegArgs {
  int L, h, hpad;
  const void* tab;        // TABLE mode: [L(L+1)/2][hpad] P̄ rows
  const int* morder;      // MFMA kernel: order run by workgroup column b (nullptr: b itself)
  const double* xs;       // RECURRENCE mode: h nodes
  const double* rcoef;    // [L(L+1)/2]
  const double* rgam;     // [L(L+1)/2]
  const double* rseed;    // [L][h]
  const double* rck;      // [nparts][4][h][2] recurrence checkpoints (row-split kernel)
  const SplitPartH* parts;// row-split kernel: work list of parts
  int nparts;
  int maxlen;             // longest part (rows)
  void* pbuf;             // [chunks][npb][IB][h][2] partial synthesis sums of cut orders (cpx<T>)
  int npb;                // partial slots per item chunk
  int item0, nb;
  const ItemDev* items;
  cpx<T>* spec;
  const T* hl;            // [nitems][hl_stride] heat multipliers (by absolute item index), + 32 readable entries
  int hl_stride;
  int mode;               // 0 fused (analysis, x h, synthesis), 1 analysis -> coeff, 2 coeff -> synthesis
  int jpt;                // RECURRENCE mode: latitude chains per thread (0 = automatic)
  cpx<T>* coeff;          // packed (m, l) coefficients, item offsets ItemDev::coff (modes 1, 2)
  long long soff0;        // spectral offset of the launch's first item (items of a launch are
                          // consecutive, 2 L h complex entries each)
};

// Launchers (kernels.hip).  All enqueue on `stream` and return the launch status.
// set_launch_events: time the next row/Legendre launch with these events.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
template <typename T>
hipError_t launch_rows(const RowArgs<T>& a, int nb, hipStream_t stream);
template <typename T>
hipError_t launch_legendre(const LegArgs<T>& a, int table_kind, int ib, hipStream_t stream);
int recur_jpt(int h);
int recur_jpt_valid(int h, int jpt);
size_t split_lds_bytes(int maxlen, int h, int ib, int real_bytes);  // maxlen: longest part (rows)
template <typename T>
hipError_t launch_legendre_split(const LegArgs<T>& a, int ib, hipStream_t stream);

// Batched MFMA Legendre GEMM (table plans): nt column tiles of 16 per workgroup.
template <typename T>
hipError_t launch_legendre_mma(const LegArgs<T>& a, int table_kind, int nt, hipStream_t stream);
size_t mma_lds_bytes(int L, int hpad, int nt, int table_kind, bool narrow = false);

template <typename T>
hipError_t launch_reduce(const RowArgs<T>& a, int nb, int nchk_done, double* res, double* ehist,
                         hipStream_t stream);
template <typename T>
hipError_t launch_gauge(const RowArgs<T>& a, int nb, int k, double* gout, hipStream_t stream);
// Per (row, item) float64 (sum a, sum a g, sum a g^2) of g = d / a; items of one
// grid, item i's field at d + foff[i] (foff device), aw[j] the float64 area
// weight of row pair j (device).  out: [items][nlat][3].
template <typename T>
hipError_t launch_row_stats(const RowArgs<T>& a, int nitems, const T* d, const long long* foff, const double* aw,
                            double* out, hipStream_t stream);
// Per item (g_k, S_A, S_B) of iteration k: gout[3 it + {0, 1, 2}].
template <typename T>
hipError_t launch_gauge3(const RowArgs<T>& a, int nb, int k, double* gout, hipStream_t stream);
template <typename T>
hipError_t launch_combine(const CombineDev* d, int npairs, long long maxn, T* out, hipStream_t stream);

// Table element kinds.
enum { TAB_F64 = 0, TAB_F32 = 1, TAB_BF16 = 2, TAB_RECUR = 3 };

// Operand forms of the recurrence-fed matrix-core Legendre kernel: float32,
// bfloat16, or split bfloat16 (hi + lo, three products).
enum { RM_F32 = 0, RM_BF16 = 1, RM_BF16X3 = 2 };
// nt column tiles of 16 (8 nt items) per workgroup, nt in {1, 2}.
template <typename T>
hipError_t launch_legendre_rmma(const LegArgs<T>& a, int op, int nt, hipStream_t stream);
size_t rmma_lds_bytes(int L, int h, int nt, int op);

}  // namespace shot
