// Slice-pair products on the INT8 matrix cores, fused with the exact
// combination of the real products and the carry chain.
//
// With A = diag(2^G) sum_s X_s 2^(-w(s+1)) and B = sum_t Y_t 2^(-w(t+1)) diag(2^H)
// (balanced base-2^8 digits in [-128, 127]), every real product is
//     X Y = diag(2^G) [ sum_d D_d 2^(-w(d+2)) ] diag(2^H),   D_d = sum_{s+t=d} X_s Y_t,
// i.e. the slice-pair products C_{alpha beta} of Algorithm 2 grouped by
// anti-diagonal d = s + t.  Each D_d is an exact integer matrix: products of
// digits are at most 2^14 in magnitude and the planner limits the terms per
// diagonal so that int32 accumulation cannot overflow.
//
// Work of one wavefront: a 16 x 16 output tile (v_mfma_i32_16x16x64_i8) and a
// contraction chunk.  The diagonals are processed in bands of W consecutive
// diagonals [d0, d0 + W), least significant band first, with one int32
// accumulator per diagonal (and per real product).  A band is worked in units
// (band, pass, 64-wide k-block); inside a unit the wave walks s upward and the
// B fragments Y_t with s + t in the band form a sliding window of W registers
// (a ring: the fragment loaded at step v enters slot v mod W), so each step
// needs one A fragment X_s and one new B fragment Y_{d0-s} and issues W MFMAs
// (every pair (s, t) of the band exactly once).  Only a unit whose walk
// starts at s = 0 and ends short of s_hi = d0 + W - 1 begins with W steps
// that only fill the ring; the others start on pairs outside the operands,
// whose MFMAs the first ring turn skips.  Units are padded with steps on zero
// fragments to an even number of queue entries.
//
// Operand fragments (16 rows x 64 k, 16 bytes per lane, 1 KB contiguous) stream
// from the tile-major digit planes (consecutive slices of a tile are k-rows
// apart, so the walk touches few pages: striding whole planes per step thrashes
// the TLB) into a workgroup-shared queue in LDS by direct global->LDS loads
// (16 bytes per lane: one fragment per instruction).  A queue entry holds the
// fragments of NS consecutive steps for the workgroup's 2 x 2 tiles; each
// fragment is loaded once and read by the two wavefronts that need it.  The
// four wavefronts walk the (band, pass, k-block, step pair) sequence in
// lockstep, each issuing a quarter of the loads QS - 1 entries ahead; one
// barrier per entry publishes the loads, and every wavefront reads its
// fragments from LDS one entry ahead of their use.  This keeps about QS
// entries of loads in flight without spending registers on them.  The digit
// planes carry zero slices around their digits, so no load is conditional.
//
// When a band is complete its W diagonals are combined into Re and Im
// (4M, eq. 5: the accumulators hold Re and Im directly, the B side supplying
// -Im B; 3M, eq. 6: T1, T2, T3 with Re = T1 - T2, Im = T3 - T1 - T2) and pushed,
// least significant first, through a per-element int64 carry chain that emits
// one normalised base-2^8 digit per diagonal, stored contiguously per output
// component; the final carry is the signed top of the exact result.
//
// Workgroups are 2 x 2 tiles; their order is XCD-aware so that the workgroups
// resident on one XCD cover a compact block of the output and share operand
// panels in that XCD's L2.
//
// One real product per workgroup (forms F3P and F4P, gemm_i8_p_kernel): the
// real products of a tile group run as separate work items, each with one
// accumulator set and half the LDS queue, so that two workgroups share a
// compute unit and one SIMD's second wavefront issues MFMAs while the first
// waits.  Each item's carry chain emits its product's share of Re and Im
// into a digit stream of its own (3M: T1 to Re and -Im, T2 to -Re and -Im,
// T3 to Im; 4M: Re A Re B and Im A (-Im B) to Re, Re A Im B and Im A Re B to
// Im; the digits of a component a product does not touch are not stored);
// the rounding kernel adds the streams.
#include "mpcg_internal.h"

#include <type_traits>

namespace mpcg {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

__device__ inline v4i mfma(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// s_waitcnt constraining only the vector-memory counter (gfx9 encoding: vmcnt
// in bits 3:0 and 15:14; expcnt bits 6:4 and lgkmcnt bits 11:8 left at their
// maxima).  The compiler does not relate direct-to-LDS loads to later LDS
// reads, so the queue states its own waits.
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup -> (contraction chunk, 2x2 tile group).  Blocks are dispatched to
// the 8 XCDs round-robin; consecutive blocks of one XCD get consecutive
// positions of a grouped (4 tile-group rows at a time) order.
__device__ inline void map_block(int b, int nblk, int gm, int gn, int& split, int& gi, int& gj) {
  constexpr int NXCD = 8, GROUP = 4;
  const int per = nblk / NXCD, rem = nblk % NXCD;
  const int xcd = b % NXCD, slot = b / NXCD;
  const int lin = (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  const int groups = gm * gn;
  split = lin / groups;
  const int gid = lin - split * groups;
  const int gsz = GROUP * gn;
  const int grp = gid / gsz, in = gid - grp * gsz;
  const int rows_here = min(GROUP, gm - grp * GROUP);
  gi = grp * GROUP + in % rows_here;
  gj = in / rows_here;
}

// Band geometry: diagonals [d0, d0 + W) and the s range holding its pairs.
// A band whose pairs reach s = 0 at its first diagonal and t = 0 at its last
// (s_lo = 0, s_hi = d0 + W - 1) is walked downward from s_hi: its ring then
// starts on pairs with t < 0 (known zeros, skipped) and it ends at s = 0
// with no pair outside the operands.  The others are walked upward.  Down
// bands are the most significant ones (a suffix of the band order).
__host__ __device__ inline bool band_down(int d0, int W, int SA, int SB) {
  return d0 <= SB - 1 && d0 + W - 1 <= SA - 1;
}

struct Band {
  int d0, s_lo, s_hi;
  bool down;
  __device__ inline void set(int band, int W, int Dmax, int SA, int SB) {
    d0 = Dmax + 1 - W * (band + 1);
    s_lo = max(0, d0 - (SB - 1));
    s_hi = min(SA - 1, d0 + W - 1);
    down = band_down(d0, W, SA, SB);
  }
};

// 16-digit chunks per output component: the bands cover digits q = Dmax - d
// for q < W * nbands.
__host__ __device__ inline int digit_chunks(int Dmax, int W) {
  const int nbands = (Dmax + W) / W;
  return (nbands * W + 15) / 16;
}

// Compile-time shape of the fragment queue.  An entry holds NS consecutive
// steps; per step: the A fragment X_s of the workgroup's two row tiles and the
// B fragments Y_{d0-s} of its two column tiles for each B plane.
template <int W, int F>
struct Q {
  static constexpr int NS = (W % 8 == 0) ? 4 : 2;  // steps per entry (a ring turn is an even number of entries)
  static constexpr int NB = F == F4M ? 2 : 1;  // B planes per step
  static constexpr int E = 2 + 2 * NB;      // fragments per step
  static constexpr int ENT = NS * E;        // fragments per entry
  static constexpr int PW = ENT / 4;        // loads each wavefront issues per entry
  static constexpr int QS = ((F == F3P || F == F4P) ? 80 : 160) / ENT;  // entries in the queue (160 KB of LDS; 80 KB
                                                          // for two workgroups per compute unit)
  static constexpr int VM = (QS - 3) * PW;  // own loads still allowed in flight when the next entry must have landed
  static constexpr int VM0 = (QS - 2) * PW; // the same for entry 0 after the prologue
  static constexpr int NPASS = (F == F3M || F == F3P) ? 3 : (F == F4P ? 4 : 2);
  static constexpr int NACC = F == F3M ? 3 : ((F == F3P || F == F4P) ? 1 : 2);
  static constexpr int CH = W / NS;         // entries per chunk (W steps: one turn of the ring)
  static_assert(CH % 2 == 0, "entries alternate between two register buffers");
  static_assert(VM0 < 64, "vmcnt range");
};

// Steps of a unit (band, pass, k-block): upward from s_lo > 0, s from s_lo to
// s_hi (the first ring turn skips the slots not yet written: their pairs have
// t > S_B - 1); upward from s_lo = 0, s from -W (the first W steps only fill
// the ring) to s_hi; downward, s from s_hi to 0; padded with steps on zero
// fragments to an even number of entries of NS steps.
__device__ inline int unit_entries(const Band& g, int W, int NS) {
  const int n = g.down ? g.s_hi + 1 : (g.s_lo > 0 ? g.s_hi - g.s_lo + 1 : g.s_hi - (g.s_lo - W) + 1);
  const int per = 2 * NS;
  return (n + per - 1) / per * 2;
}

// Zero slices around each digit plane.  An upward unit reads X_s for s in
// [s_lo - W, s_hi + 2 NS - 1] and Y_t for t = d0 - s, i.e. t in
// [2 - W - 2 NS, S_B - 1 + W]; a downward unit reads X_s for s in
// [1 - 2 NS, s_hi] and Y_t for t in [0, S_B + W + 2 NS - 3].  That many
// zero slices lie below and above each plane's S digits (the host lays the
// planes out so that one run of max(lo, hi) zero slices serves as a plane's
// upper and the next plane's lower pad), so that every load of a unit is
// unconditional and the pairs outside the operands multiply zeros.
__host__ __device__ inline void pads_for(int W, int& alo, int& ahi, int& blo, int& bhi) {
  const int NS = (W % 8 == 0) ? 4 : 2;
  alo = W;
  ahi = 2 * NS - 1;
  blo = W + 2 * NS - 2;
  bhi = W + 2 * NS - 2;
}

// This wavefront's share of the loads, walking the (band, pass, k-block,
// entry) sequence.  Load i of an entry is fragment f = wv * PW + i: the A
// fragment of row tile c or a B fragment of column tile c, of step h of the
// entry.  Within a unit its (wave-uniform) source moves by a constant stride
// per entry, so a load costs a 64-bit scalar add and the instruction itself;
// only the end of a unit branches.
template <int W, int F>
struct Producer {
  using G = Q<W, F>;
  static constexpr int PW = G::PW;
  size_t xplane, yplane;  // bytes between consecutive slices of a tile's plane
  int SA, SB, Dmax, nbands, kb0, kb1;
  int xs, ys, xlo, ylo;   // slices per plane (with pads) and lower pads
  unsigned lane16;
  // per load (static index i)
  const int8_t* tb[PW];   // the tile's planes (wave-uniform)
  int isa[PW], hh[PW], sel[PW], foff[PW];
  // walk state (the passes of a unit run over [pass_lo, pass_hi))
  int band, pass, kb, e, ne, pass_lo, pass_hi;
  Band g;
  bool done;
  const int8_t* src[PW];
  int64_t dlt[PW];

  __device__ inline void share(int wv, const int8_t* X0, const int8_t* X1, const int8_t* Y0, const int8_t* Y1) {
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      const int f = wv * PW + i;
      const int h = f / G::E, x = f - h * G::E;
      const int a = x < 2 ? 1 : 0;
      const int c = a ? x : ((x - 2) & 1);
      tb[i] = a ? (c ? X1 : X0) : (c ? Y1 : Y0);
      isa[i] = a;
      hh[i] = h;
      sel[i] = a ? 0 : ((x - 2) >> 1);
      foff[i] = f * 1024;
    }
  }

  // set sources and strides for the unit (band, pass, kb)
  __device__ inline void unit_begin() {
    ne = unit_entries(g, W, G::NS);
    e = 0;
    // step h of entry e: s = s0 + dir (NS e + h), t = t0 - dir (NS e + h)
    const int dir = g.down ? -1 : 1;
    const int s0 = g.down ? g.s_hi : (g.s_lo > 0 ? g.s_lo : g.s_lo - W);
    const int t0 = g.down ? g.d0 + W - 1 - g.s_hi : g.d0 - s0;
    int pa, pb0, pb1;
    if (F == F4P) {  // Re Re, Im (-Im) into Re; Re Im, Im Re into Im
      pa = pass & 1; pb0 = pass == 1 ? 2 : (pass == 2 ? 1 : 0); pb1 = 0;
    } else if (F != F4M) {  // X plane p with Y plane p
      pa = pass; pb0 = pass; pb1 = 0;
    } else {  // Re A with (Re B, Im B); Im A with (-Im B, Re B)
      pa = pass; pb0 = pass == 0 ? 0 : 2; pb1 = pass == 0 ? 1 : 0;
    }
    const int64_t ko = (int64_t)kb * 1024;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      const int h = hh[i];
      if (isa[i]) {
        src[i] = tb[i] + ((int64_t)(pa * xs + xlo + s0 + dir * h) * (int64_t)xplane + ko);
        dlt[i] = dir * G::NS * (int64_t)xplane;
      } else {
        const int pl = sel[i] ? pb1 : pb0;
        src[i] = tb[i] + ((int64_t)(pl * ys + ylo + t0 - dir * h) * (int64_t)yplane + ko);
        dlt[i] = -dir * G::NS * (int64_t)yplane;
      }
    }
  }
  __device__ inline void start(int band0) {
    band = band0;
    pass = pass_lo;
    kb = kb0;
    g.set(band0, W, Dmax, SA, SB);
    done = false;
    unit_begin();
  }
  __device__ inline void next_unit() {
    if (++kb >= kb1) {
      kb = kb0;
      if (++pass >= pass_hi) {
        pass = pass_lo;
        if (++band >= nbands) {
          // past the end: keep reloading the tile's first fragment (never consumed)
          done = true;
          ne = 0x7fffffff;
#pragma unroll
          for (int i = 0; i < PW; ++i) {
            src[i] = tb[i];
            dlt[i] = 0;
          }
          return;
        }
        g.set(band, W, Dmax, SA, SB);
      }
    }
    unit_begin();
  }
  // load i of the current entry into the entry at `dst`
  __device__ inline void issue(int i, int8_t* dst) const {
    __builtin_amdgcn_global_load_lds(src[i] + lane16, (lds_void*)(dst + foff[i]), 16, 0, 0);
  }
  __device__ inline void step() {
#pragma unroll
    for (int i = 0; i < PW; ++i) src[i] += dlt[i];
  }
  __device__ inline void tail() {
    if (__builtin_expect(++e >= ne, 0)) next_unit();
  }
};

template <int W, int F>
struct Consumer {
  using G = Q<W, F>;
  static_assert(W % 4 == 0, "a ring turn is an even number of entries");
  static constexpr int NB = G::NB, E = G::E, QS = G::QS, NACC = G::NACC, PW = G::PW;
  int8_t* q;  // the workgroup's queue: QS entries of ENT KB
  int lane, wi, wj;
  int slot;   // queue entry of the current steps
  static constexpr int NS = G::NS;
  // fragments of the current entry (parity p) and of the next one (parity 1 - p)
  v4i abuf[2][NS], bbuf[2][NS][NB];
  v4i ring0[W], ring1[F == F4M ? W : 1];

  template <int P>
  __device__ inline void read(int sl) {
#pragma unroll
    for (int h = 0; h < NS; ++h) {
      const int8_t* base = q + (sl * G::ENT + h * E) * 1024 + lane * 16;
      abuf[P][h] = *reinterpret_cast<const v4i*>(base + wi * 1024);
#pragma unroll
      for (int p = 0; p < NB; ++p) bbuf[P][h][p] = *reinterpret_cast<const v4i*>(base + (2 + 2 * p + wj) * 1024);
    }
  }

  // One entry: ring steps V = NS C .. NS C + NS - 1 (V mod W static).  Once
  // this wavefront's loads of the next entry have landed, the barrier makes
  // everybody's loads of it visible (it is read into the other register
  // buffer) and tells that every wavefront has used the previous entry, whose
  // queue slot is then refilled by loads spread between the MFMAs.
  // RAMP: the first ring turn of a ramped unit; at its step V the ring slots
  // V + 1 .. W - 1 steps old have not been written (their pairs are known
  // zeros), so those MFMAs are skipped.  DOWN: a downward unit, whose ring
  // slot jj steps old holds the B fragment of diagonal d0 + W - 1 - jj.
  template <int C, bool MF, int Q0, int Q1, bool RAMP = false, bool DOWN = false>
  __device__ inline void entry(v4i (&acc)[NACC][W], Producer<W, F>& P) {
    constexpr int PAR = C & 1;
    wait_vmcnt<G::VM>();
    __builtin_amdgcn_s_barrier();
    int8_t* dst = q + (slot == 0 ? QS - 1 : slot - 1) * G::ENT * 1024;
    read<1 - PAR>(slot + 1 == QS ? 0 : slot + 1);
#pragma unroll
    for (int h = 0; h < NS; ++h) {
      constexpr int V0 = NS * C;
      const int V = V0 + h;
      ring0[V % W] = bbuf[PAR][h][0];
      if (F == F4M) ring1[V % W] = bbuf[PAR][h][NB - 1];
      // in accumulator order: the same accumulator recurs only W MFMAs later,
      // also across steps
#pragma unroll
      for (int j = 0; j < W; ++j) {
        if (MF && (!RAMP || j <= V)) {
          const int r = (V - j + W) % W;      // ring slot of the fragment loaded j steps ago
          const int ja = DOWN ? W - 1 - j : j;  // its diagonal d0 + ja
          acc[Q0][ja] = mfma(abuf[PAR][h], ring0[r], acc[Q0][ja]);
          if (F == F4M) acc[Q1][ja] = mfma(abuf[PAR][h], ring1[r], acc[Q1][ja]);
        }
        // spread this wavefront's loads over the entry
        constexpr int per = (PW + NS - 1) / NS;
        const int i = h * per + j;
        if (j < per && i < PW) P.issue(i, dst);
      }
    }
    P.step();
    slot = slot + 1 == QS ? 0 : slot + 1;
    P.tail();
  }

  template <int C, bool MF, int Q0, int Q1, bool RAMP = false, bool DOWN = false>
  __device__ inline void chunk(v4i (&acc)[NACC][W], Producer<W, F>& P, int left) {
    if constexpr (C < G::CH) {
      if (MF && left <= C) return;
      entry<C, MF, Q0, Q1, RAMP, DOWN>(acc, P);
      chunk<C + 1, MF, Q0, Q1, RAMP, DOWN>(acc, P, left);
    }
  }

  // One unit.  KIND 0: upward from s_lo > 0, a ramped first turn (its pairs
  // with t >= S_B are known zeros); 1: upward from s_lo = 0, a chunk of
  // ring-filling entries first; 2: downward, a ramped first turn (pairs with
  // t < 0).  Then chunks with MFMAs.
  template <int Q0, int Q1, int KIND>
  __device__ inline void unit(v4i (&acc)[NACC][W], Producer<W, F>& P, const Band& g) {
    const int ne = unit_entries(g, W, NS);
    if constexpr (KIND == 1) {
      chunk<0, false, Q0, Q1>(acc, P, G::CH);
    } else {
      chunk<0, true, Q0, Q1, true, KIND == 2>(acc, P, ne);
    }
    for (int e0 = G::CH; e0 < ne; e0 += G::CH) chunk<0, true, Q0, Q1, false, KIND == 2>(acc, P, ne - e0);
  }
};

// One work item: the 2 x 2 tile group (gi, gj) of stream `split`.
template <int W, int F>
__device__ __attribute__((always_inline)) inline void gemm_item(const GemmArgs& a, int split, int gi, int gj,
                                                                 int8_t* lds_queue) {
  using G = Q<W, F>;
  using C = Consumer<W, F>;
  constexpr int NACC = G::NACC;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  const int wi = wv & 1, wj = wv >> 1;
  const int ti = 2 * gi + wi;
  const int tj = 2 * gj + wj;
  const int tile = tj * a.mt + ti;
  // stream `split` = (contraction chunk c, band group g, pass p) as
  // (c bs + g) ps + p: the bands of group g only when the bands are split
  // over workgroups (bs > 1), the real product p only when the products are
  // (ps > 1)
  const int bs = a.bsplit > 1 ? a.bsplit : 1;
  const int ps = a.psplit > 1 ? a.psplit : 1;
  const int pass_sel = split % ps;
  const int kchunk = split / ps / bs;
  const int nb_all = (a.Dmax + W) / W;
  const int bpg = (nb_all + bs - 1) / bs;  // bands per group
  const int band_lo = min(nb_all, (split / ps - kchunk * bs) * bpg);
  const int band_hi = min(nb_all, band_lo + bpg);
  const int pass_lo = ps > 1 ? pass_sel : 0, pass_hi = ps > 1 ? pass_sel + 1 : G::NPASS;
  const int kbps = (a.kblocks + a.ksplit - 1) / a.ksplit;
  const int kb0 = kchunk * kbps;
  const int kb1 = min(a.kblocks, kb0 + kbps);
  if (band_lo >= band_hi) return;  // no band in this group (the host plans none such)

  Producer<W, F> P;
  // tile-major planes: consecutive slices of one tile and plane are a k-row
  // (kblocks fragments) apart, so a unit's loads stay within a few pages
  P.xplane = (size_t)a.kblocks * 1024;
  P.yplane = (size_t)a.kblocks * 1024;
  P.lane16 = (unsigned)lane * 16u;
  P.xs = a.xs;
  P.ys = a.ys;
  P.xlo = a.xlo;
  P.ylo = a.ylo;
  P.SA = a.SAp;
  P.SB = a.SBp;
  P.Dmax = a.Dmax;
  P.nbands = band_hi;
  P.kb0 = kb0;
  P.kb1 = kb1;
  P.pass_lo = pass_lo;
  P.pass_hi = pass_hi;
  {
    const size_t xtile = (size_t)((F == F3M || F == F3P) ? 3 : 2) * a.xs * a.kblocks * 1024;  // bytes of one row tile
    const size_t ytile = (size_t)3 * a.ys * a.kblocks * 1024;             // bytes of one column tile
    const int8_t* X0 = a.X + (size_t)(2 * gi) * xtile;  // row tiles 2gi, 2gi+1
    const int8_t* Y0 = a.Y + (size_t)(2 * gj) * ytile;  // column tiles 2gj, 2gj+1
    P.share(wv, X0, X0 + xtile, Y0, Y0 + ytile);
  }
  P.start(band_lo);

  C c;
  c.q = lds_queue;
  c.lane = lane;
  c.wi = wi;
  c.wj = wj;
  c.slot = 0;
  // fill entries 0 .. QS-2, then read entry 0
#pragma unroll 1
  for (int u = 0; u < G::QS - 1; ++u) {
#pragma unroll
    for (int i = 0; i < G::PW; ++i) P.issue(i, c.q + u * G::ENT * 1024);
    P.step();
    P.tail();
  }
  wait_vmcnt<G::VM0>();
  __builtin_amdgcn_s_barrier();
  c.template read<0>(0);

  int64_t cre[4], cim[4];
  int32_t lre[4], lim[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cre[r] = cim[r] = 0;
    lre[r] = lim[r] = -1;
  }
  // this lane's digit bytes: [split][tile][slot 8][chunk][lane][16]
  const int nchunk = digit_chunks(a.Dmax, W);
  const size_t slot_stride = (size_t)nchunk * 1024;
  // (a wave-uniform base and 32-bit per-lane offsets: no 64-bit address per
  // store stays live across the band loop)
  uint8_t* dig = reinterpret_cast<uint8_t*>(a.digits) + (size_t)(split * a.mt * a.nt + tile) * 8 * slot_stride;
  const uint32_t dig_lane = (uint32_t)lane * 16u;

  // One band: its units, then the carry chain over its W diagonals.
  auto band_body = [&](const int band, auto kind_tag) {
    constexpr int KIND = decltype(kind_tag)::value;
    Band g;
    g.set(band, W, a.Dmax, a.SAp, a.SBp);
    v4i acc[NACC][W];
#pragma unroll
    for (int p = 0; p < NACC; ++p)
#pragma unroll
      for (int j = 0; j < W; ++j) acc[p][j] = v4i{0, 0, 0, 0};

    // the passes [pass_lo, pass_hi) of this work item (all of them unless
    // the real products run on workgroups of their own; the others' sums
    // then stay zero, and the carry chain below emits this pass's share)
    if constexpr (F == F3M) {  // T1 = Re Re, T2 = Im Im, T3 = (Re+Im)(Re+Im)
      if (pass_lo <= 0)
#pragma unroll 1
        for (int kb = kb0; kb < kb1; ++kb) c.template unit<0, 0, KIND>(acc, P, g);
      if (pass_lo <= 1 && 1 < pass_hi)
#pragma unroll 1
        for (int kb = kb0; kb < kb1; ++kb) c.template unit<1, 1, KIND>(acc, P, g);
      if (2 < pass_hi)
#pragma unroll 1
        for (int kb = kb0; kb < kb1; ++kb) c.template unit<2, 2, KIND>(acc, P, g);
    } else if constexpr (F == F3P || F == F4P) {  // this work item's one real product
#pragma unroll 1
      for (int kb = kb0; kb < kb1; ++kb) c.template unit<0, 0, KIND>(acc, P, g);
    } else if constexpr (F == FSEP) {  // T1 = X0 Y0 and T2 = X1 Y1, kept apart
      if (pass_lo <= 0)
#pragma unroll 1
        for (int kb = kb0; kb < kb1; ++kb) c.template unit<0, 0, KIND>(acc, P, g);
      if (1 < pass_hi)
#pragma unroll 1
        for (int kb = kb0; kb < kb1; ++kb) c.template unit<1, 1, KIND>(acc, P, g);
    } else {  // Re += ReA ReB + ImA (-ImB),  Im += ReA ImB + ImA ReB
#pragma unroll 1
      for (int pass = pass_lo; pass < pass_hi; ++pass)
#pragma unroll 1
        for (int kb = kb0; kb < kb1; ++kb) c.template unit<0, 1, KIND>(acc, P, g);
    }
    // the band is complete: push its diagonals through the carry chains, least
    // significant first; digit q = Dmax - d of component slot k goes to
    // digits[k][q / 16][lane][q % 16]: each output component's digits are
    // contiguous in 16-digit chunks (one 16-byte word per lane and chunk)
    uint32_t wre[4][W / 4], wim[4][W / 4];
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
      const int j = W - 1 - jj;  // q = W band + jj
      const int d = g.d0 + j;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t vre, vim;
        if constexpr (F == F3M) {
          const int64_t t1 = acc[0][j][r], t2 = acc[1][j][r], t3 = acc[2][j][r];
          vre = t1 - t2;
          vim = t3 - t1 - t2;
        } else if constexpr (F == F3P) {  // T1: (+, -), T2: (-, -), T3: (0, +)
          const int64_t t = acc[0][j][r];
          vre = pass_lo == 0 ? t : (pass_lo == 1 ? -t : 0);
          vim = pass_lo == 2 ? t : -t;
        } else if constexpr (F == F4P) {  // Re: products 0, 1; Im: 2, 3
          const int64_t t = acc[0][j][r];
          vre = pass_lo < 2 ? t : 0;
          vim = pass_lo < 2 ? 0 : t;
        } else {
          vre = acc[0][j][r];
          vim = acc[1][j][r];
        }
        uint32_t dre = 0, dim = 0;
        if (d >= 0) {  // diagonals below 0 (the last band's overhang) are empty
          cre[r] += vre;
          cim[r] += vim;
          dre = (uint32_t)(cre[r] & ((1 << I8_W) - 1));
          dim = (uint32_t)(cim[r] & ((1 << I8_W) - 1));
          cre[r] >>= I8_W;
          cim[r] >>= I8_W;
          if (dre && lre[r] < 0) lre[r] = d;
          if (dim && lim[r] < 0) lim[r] = d;
        }
        if (jj % 4 == 0) {
          wre[r][jj / 4] = dre;
          wim[r][jj / 4] = dim;
        } else {
          wre[r][jj / 4] |= dre << (8 * (jj % 4));
          wim[r][jj / 4] |= dim << (8 * (jj % 4));
        }
      }
    }
    // (T3 adds nothing to Re, a 4M product to one component only: the other
    // digits of its stream are neither written nor read)
    const bool keep_re = F == F3P ? pass_lo != 2 : (F == F4P ? pass_lo < 2 : true);
    const bool keep_im = F == F4P ? pass_lo >= 2 : true;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int u = 0; u < W / 4; ++u) {
        const int q = W * band + 4 * u;
        const uint32_t at = (uint32_t)(q >> 4) * 1024u + (uint32_t)(q & 15) + dig_lane;
        if (keep_re) *reinterpret_cast<uint32_t*>(dig + ((uint32_t)r * (uint32_t)slot_stride + at)) = wre[r][u];
        if (keep_im) *reinterpret_cast<uint32_t*>(dig + ((uint32_t)(4 + r) * (uint32_t)slot_stride + at)) = wim[r][u];
      }
  };
  // least significant first: upward bands with s_lo > 0, the upward band(s)
  // from s_lo = 0 that stop short of d0 + W - 1, then the downward ones (each
  // class is a contiguous run of the band order)
  // a band group's stream: zeros from the start of the 16-digit chunk holding
  // its first digit (the other groups' digits are not in this stream)
  for (int q = (W * band_lo) & ~15; q < W * band_lo; q += 4) {
    const uint32_t at = (uint32_t)(q >> 4) * 1024u + (uint32_t)(q & 15) + dig_lane;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      *reinterpret_cast<uint32_t*>(dig + ((uint32_t)r * (uint32_t)slot_stride + at)) = 0u;
      *reinterpret_cast<uint32_t*>(dig + ((uint32_t)(4 + r) * (uint32_t)slot_stride + at)) = 0u;
    }
  }
  int band = band_lo;
#pragma unroll 1
  for (; band < P.nbands && a.Dmax + 1 - W * (band + 1) > a.SBp - 1 &&
         !band_down(a.Dmax + 1 - W * (band + 1), W, a.SAp, a.SBp); ++band)
    band_body(band, std::integral_constant<int, 0>{});
#pragma unroll 1
  for (; band < P.nbands && !band_down(a.Dmax + 1 - W * (band + 1), W, a.SAp, a.SBp); ++band)
    band_body(band, std::integral_constant<int, 1>{});
#pragma unroll 1
  for (; band < P.nbands; ++band) band_body(band, std::integral_constant<int, 2>{});
  // a band group's stream: zeros to the end of the chunk holding its last
  // digit; its carry into the next group's digits is left in `top`
  for (int q = W * band_hi; q < ((W * band_hi + 15) & ~15); q += 4) {
    const uint32_t at = (uint32_t)(q >> 4) * 1024u + (uint32_t)(q & 15) + dig_lane;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      *reinterpret_cast<uint32_t*>(dig + ((uint32_t)r * (uint32_t)slot_stride + at)) = 0u;
      *reinterpret_cast<uint32_t*>(dig + ((uint32_t)(4 + r) * (uint32_t)slot_stride + at)) = 0u;
    }
  }
  // the producer ran past the end of the stream: drain its loads before the LDS is released
  wait_vmcnt<0>();

  const size_t ob = ((size_t)(split * a.mt * a.nt + tile) * 64 + lane) * 8;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a.top[ob + r] = cre[r];
    a.top[ob + 4 + r] = cim[r];
    a.lnz[ob + r] = lre[r];
    a.lnz[ob + 4 + r] = lim[r];
  }
}

template <int W, int F>
__global__ __launch_bounds__(256) void gemm_i8_kernel(GemmArgs a) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds_queue[];
  int split, gi, gj;
  map_block(blockIdx.x, gridDim.x, a.mt >> 1, a.nt >> 1, split, gi, gj);
  gemm_item<W, F>(a, split, gi, gj, lds_queue);
}

// Persistent form for a batch of products: block b works through its list of
// items (problem, gi, gj, split), the lists balanced by the host
// (longest-processing-time first).  The queue is drained at the end of an
// item; the barrier keeps a fast wavefront from refilling it while another
// still reads the previous item's last entry.
template <int W, int F>
__global__ __launch_bounds__(256) void gemm_i8_batched_kernel(const GemmArgs* __restrict__ probs,
                                                              const int4* __restrict__ items,
                                                              const int* __restrict__ first) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds_queue[];
  const int i0 = first[blockIdx.x], i1 = first[blockIdx.x + 1];
  for (int i = i0; i < i1; ++i) {
    const int4 it = items[i];
    const GemmArgs a = probs[it.x];
    gemm_item<W, F>(a, it.w, it.y, it.z, lds_queue);
    __syncthreads();
  }
}

// One real product per work item: a third of the registers, half the queue,
// two workgroups per compute unit.
template <int W, int F>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void gemm_i8_p_kernel(GemmArgs a) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds_queue[];
  int split, gi, gj;
  map_block(blockIdx.x, gridDim.x, a.mt >> 1, a.nt >> 1, split, gi, gj);
  gemm_item<W, F>(a, split, gi, gj, lds_queue);
}

template <int W, int F>
hipError_t launch_wm(const GemmArgs& a, hipStream_t stream) {
  using G = Q<W, F>;
  const int blocks = (a.mt / 2) * (a.nt / 2) * a.ksplit * (a.bsplit > 1 ? a.bsplit : 1) * (a.psplit > 1 ? a.psplit : 1);
  const size_t lds = (size_t)G::QS * G::ENT * 1024;
  if constexpr (F == F3P || F == F4P) {
    hipError_t e = hipFuncSetAttribute((const void*)gemm_i8_p_kernel<W, F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    gemm_i8_p_kernel<W, F><<<dim3(blocks), dim3(256), lds, stream>>>(a);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)gemm_i8_kernel<W, F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    gemm_i8_kernel<W, F><<<dim3(blocks), dim3(256), lds, stream>>>(a);
  }
  return hipGetLastError();
}

template <int W>
hipError_t launch_w(const GemmArgs& a, hipStream_t stream) {
  switch (a.form) {
    case F4M: return launch_wm<W, F4M>(a, stream);
    case F3M: return launch_wm<W, F3M>(a, stream);
    case FSEP: return launch_wm<W, FSEP>(a, stream);
    case F3P:  // one real product per workgroup (20-wide bands do not fit two workgroups' registers)
      if constexpr (W <= 16) {
        if (a.psplit == 3 && a.bsplit <= 1) return launch_wm<W, F3P>(a, stream);
      }
      return hipErrorInvalidValue;
    case F4P:
      if constexpr (W <= 16) {
        if (a.psplit == 4 && a.bsplit <= 1) return launch_wm<W, F4P>(a, stream);
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int W, int F>
hipError_t launch_batched_wm(const GemmArgs* probs, const int4* items, const int* first, int blocks,
                             hipStream_t stream) {
  using G = Q<W, F>;
  const size_t lds = (size_t)G::QS * G::ENT * 1024;
  hipError_t e = hipFuncSetAttribute((const void*)gemm_i8_batched_kernel<W, F>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  gemm_i8_batched_kernel<W, F><<<dim3(blocks), dim3(256), lds, stream>>>(probs, items, first);
  return hipGetLastError();
}

template <int W>
hipError_t launch_batched_w(const GemmArgs* probs, const int4* items, const int* first, int blocks, int mode3m,
                            hipStream_t stream) {
  return mode3m ? launch_batched_wm<W, F3M>(probs, items, first, blocks, stream)
                : launch_batched_wm<W, F4M>(probs, items, first, blocks, stream);
}

}  // namespace

void gemm_i8_pads(int band, int* alo, int* ahi, int* blo, int* bhi) { pads_for(band, *alo, *ahi, *blo, *bhi); }
int gemm_i8_digit_chunks(int Dmax, int band) { return digit_chunks(Dmax, band); }

hipError_t launch_gemm_i8(const GemmArgs& a, int band, hipStream_t stream) {
  switch (band) {
    case 8: return launch_w<8>(a, stream);
    case 12: return launch_w<12>(a, stream);
    case 16: return launch_w<16>(a, stream);
    case 20: return launch_w<20>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm_i8_batched(const GemmArgs* probs, const int4* items, const int* first, int blocks,
                                  int band, int mode3m, hipStream_t stream) {
  if (blocks <= 0) return hipSuccess;
  switch (band) {
    case 8: return launch_batched_w<8>(probs, items, first, blocks, mode3m, stream);
    case 12: return launch_batched_w<12>(probs, items, first, blocks, mode3m, stream);
    case 16: return launch_batched_w<16>(probs, items, first, blocks, mode3m, stream);
    case 20: return launch_batched_w<20>(probs, items, first, blocks, mode3m, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mpcg
