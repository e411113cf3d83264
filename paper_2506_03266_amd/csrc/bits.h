// bits.h -- bit-sliced kernels for the first decoder steps (gfx950): the
// whole lattice in one workgroup at L = 64, 128 and 256 (k_bits), and
// 256 x 256 regions with halos above 256 (k_bits_tile, at the end).
//
// Registers hold emission times (see engine.h), and during the first ten
// decoder steps every emission time is at most 3 * 10 = 30: a register fits
// in 5 bits (in 2, 3 and 4 bits during the first, second and third to fifth
// steps).  Stored as bit planes -- one 32-bit word holds one bit of one
// register for 32 consecutive rows of one column -- the whole state of an
// L = 256 torus is 256 x 256 sites x 4 registers x 5 bits = 160 KiB, which a
// workgroup of four waves keeps in VGPRs.  These steps then need no halo
// (the torus wraps inside the workgroup) and no HBM state, a sample leaves
// as soon as it has no anyon, and the update works on 32 sites per
// instruction:
//
//  * Rule A^{(D)} of Def. "message passing automaton, general dimensions" in
//    emission-time form is e'(r) = max over the 3-site line C of
//    (sigma_q ? s : e_q).  The fold (anyon sites emit at the sub-step time
//    s) is one select per plane; the 3-wide maximum of B-bit values is a
//    most-significant-bit-first candidate filter (6B - 5 bitwise operations
//    for 32 sites).
//  * The move decision of eq. (degbreak) with the reading of engine.h (the
//    largest emission time wins; ties in the order -y, -x, +x, +y; no move
//    when the opposite register on that axis ties) is the same filter over
//    the four registers of a site.
//  * The feedback of eq. (ddfeedback) (a link flips iff one endpoint moves
//    across it) and the syndrome update are bitwise on the masks.
//
// Layout: wave v holds rows 64v .. 64v + 63, lane i columns CPL i .. CPL i + CPL - 1;
// word w of a column covers rows 64v + 32w .. + 31 (bit r = row 64v + 32w + r).
// Vertical neighbours inside a lane are funnel shifts (v_alignbit); across
// waves the edge rows travel through LDS packed up to 20 to a word, once per
// sub-step (one barrier).  Horizontal neighbours are in the lane or one
// wave-wide DPP rotation away (the wrap in x).
//
// Smaller tori take fewer waves and columns per lane (L = 64: one wave, one
// column per lane; L = 128: two waves, two columns per lane).
//
// At L = 256 a sample that still holds anyons after its steps leaves its
// state in the band path's HBM layout (packed u16 emission times, 16-row
// syndrome masks), from which the band kernels continue exactly.  At L = 64
// and 128 a decode that ends inside the steps writes its results here; the
// others are marked (T_dec = -1) and decoded again from their seeds by the
// whole-lattice kernel, which needs no workspace.
#pragma once

#include "band.h"

namespace mpd {

// A sample of side L = 64 CPL takes NW = CPL waves of 64 rows, each lane CPL
// columns: CPL = 1, 2, 4 for L = 64, 128, 256.
constexpr int BITS_L = 256;
constexpr int BITS_PLANES = 5;       // bit planes per register
constexpr int BITS_MAX_STEPS = 10;   // emission times <= 30 fit in 5 bits

struct BitsArgs {
  const uint64_t *seeds;
  int T_max;             // L = 64, 128: the decode's step budget
  int32_t *T_dec;        // L = 64, 128: outputs of decodes that end inside the steps
  uint8_t *flags;
  uint32_t *syn;         // final syndrome bitmaps (may be null)
  uint64_t thr;          // flip threshold floor(p 2^32) when p_arr == nullptr
  const double *p_arr;   // per-sample noise strength or nullptr
  int k;                 // decoder steps at most (<= BITS_MAX_STEPS and <= T_max)
  uint4 *E;              // band layout [n][L][L/2] register pairs (samples with anyons left)
  uint2 *S;              // band layout [n][L/16][L/2] syndrome masks
  uint32_t *alive;       // per sample: bit 0 anyons at the start, bit j anyons after step j
  uint32_t *wind;        // per sample: Wx(E), Wy(E), Wx(C), Wy(C)
  int *zero_count;       // survivor counter of the following compaction (cleared here)
  const int32_t *order;  // sample of workgroup b: order[b] (nullptr: b) -- the processing order
  const uint2 *S_in;     // syndrome in the band layout drawn by the noise kernel (its error
                         // windings already in wind), or nullptr: draw the noise here
};

// Bit planes of one register field, most significant plane last.
struct V4 {
  uint32_t p[BITS_PLANES];
};

// Site-wise maximum of three B-bit fields (planes B .. 3 are zero): the
// planes from the top, keeping per operand a mask of the sites where it
// still equals the running maximum.
template <int B>
__device__ __forceinline__ V4 max3v(const V4 &a, const V4 &b, const V4 &c) {
  V4 r;
  r.p[B - 1] = a.p[B - 1] | b.p[B - 1] | c.p[B - 1];
  uint32_t ka = a.p[B - 1] | ~r.p[B - 1], kb = b.p[B - 1] | ~r.p[B - 1], kc = c.p[B - 1] | ~r.p[B - 1];
#pragma unroll
  for (int q = B - 2; q >= 0; --q) {
    r.p[q] = (a.p[q] & ka) | (b.p[q] & kb) | (c.p[q] & kc);
    if (q > 0) {
      ka &= a.p[q] | ~r.p[q];
      kb &= b.p[q] | ~r.p[q];
      kc &= c.p[q] | ~r.p[q];
    }
  }
#pragma unroll
  for (int q = B; q < BITS_PLANES; ++q) r.p[q] = 0u;
  return r;
}

__device__ __forceinline__ uint32_t fshr(uint32_t hi, uint32_t lo, uint32_t s) {
  return __builtin_amdgcn_alignbit(hi, lo, s);  // ({hi, lo} >> s)[31:0]
}

// A copy of x that the compiler cannot see through: values derived from it
// are formed where they are used instead of being hoisted (and kept live)
// ahead of a long stretch of code.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}
// The lane's index, formed where it is used (mbcnt), so that no address
// derived from it stays live across the decoder steps.
__device__ __forceinline__ int lane_here() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}
__device__ __forceinline__ uint32_t opaque_s(uint32_t x) {  // the same for a uniform value
  asm volatile("" : "+s"(x));
  return x;
}

// m = 2 m + [x < t] in two instructions: the comparison leaves the bit in
// VCC and an add with carry shifts it in (the compiler would take three:
// compare, select, shift-or).  t is uniform.
__device__ __forceinline__ void shift_in_below(uint32_t &m, uint32_t x, uint32_t t) {
  asm("v_cmp_gt_u32 vcc, %2, %1\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc" : "+v"(m) : "v"(x), "s"(t) : "vcc");
}

// Parity over the wave's lanes of each of the low four bits of x (uniform:
// the winding bits are kept per wave, not per lane).
__device__ __forceinline__ uint32_t wave_parity4(uint32_t x) {
  uint32_t r = 0u;
#pragma unroll
  for (int b = 0; b < 4; ++b) r |= ((uint32_t)__popcll(__ballot((x >> b) & 1u)) & 1u) << b;
  return r;
}

// The value of lane i ^ 1 (DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ uint32_t swap_pair(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
}

template <int CPL>
struct BitsLane {
  uint32_t E[4][BITS_PLANES][CPL][2];  // [register: +x, -x, +y, -y][bit][column][word]
  uint32_t S[CPL][2];        // syndrome (anyon = 1)
};

// Edge rows of other waves, packed one bit per (register, plane, column) in
// the order they are used: `top` is consumed from bit 31 (then shifted
// left), `bot` from bit 0 (then shifted right).
struct Carry {
  uint32_t top, bot;
  __device__ __forceinline__ uint32_t take_top() {  // a word whose bit 31 is the next item
    const uint32_t w = top;
    top <<= 1;
    return w;
  }
  __device__ __forceinline__ uint32_t take_bot() {  // a word whose bit 0 is the next item
    const uint32_t w = bot;
    bot >>= 1;
    return w;
  }
};

// Vertical maximum over rows y - 1, y, y + 1 of register d, column c (B
// planes): r0/r1 for words 0/1.  The row below word 0 and the row above word
// 1 come from the neighbour waves through `cr`.
template <int B, int CPL>
__device__ __forceinline__ void bits_vmax(const BitsLane<CPL> &s, int d, int c, Carry &cr, V4 &r0, V4 &r1) {
  V4 x0, x1, dn, up;
#pragma unroll
  for (int q = 0; q < BITS_PLANES; ++q) {
    x0.p[q] = s.E[d][q][c][0];
    x1.p[q] = s.E[d][q][c][1];
  }
#pragma unroll
  for (int q = 0; q < B; ++q) {
    dn.p[q] = fshr(x0.p[q], cr.take_top(), 31);  // row y - 1
    up.p[q] = fshr(x1.p[q], x0.p[q], 1);         // row y + 1
  }
  r0 = max3v<B>(dn, x0, up);
#pragma unroll
  for (int q = 0; q < B; ++q) {
    dn.p[q] = fshr(x1.p[q], x0.p[q], 31);
    up.p[q] = fshr(cr.take_bot(), x1.p[q], 1);
  }
  r1 = max3v<B>(dn, x1, up);
}

// One application of A^{(D)} at sub-step time ss to the whole lattice, with
// every emission time below 2^B.  XS: this sub-step's exchange slots
// [wave][2][64]: slot 0 carries a wave's top row to the wave above (+x
// planes, -x planes, +y row maxima), slot 1 its bottom row to the wave below
// (+x, -x, -y row maxima).  Each word holds its items in the order the
// receiving wave uses them: +x columns 3 .. 0 and -x columns 0 .. 3 (the
// order of the vertical maxima), ±y columns inside planes.
template <int B, int CPL, bool TORUS>
__device__ __forceinline__ void bits_substep(BitsLane<CPL> &s, uint32_t ss, uint4 *XS, int v, int vdn, int vup,
                                             int lane) {
  constexpr int N = B * CPL;  // items per word
  // anyon sites emit now: their registers read ss
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const uint32_t M = ((ss >> q) & 1u) ? ~0u : 0u;
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int w = 0; w < 2; ++w)  // S ? M : E (one v_bitop3; M is uniform)
          s.E[d][q][c][w] = __builtin_amdgcn_bitop3_b32(M, s.E[d][q][c][w], s.S[c][w], 0xE4);
  }

  // ±x edge rows for the neighbour waves (folded values, before the update);
  // a word shifted in at bit 0 (top rows) or at bit 31 (bottom rows)
  uint32_t upx = 0u, dpx = 0u, umx = 0u, dmx = 0u, upy = 0u, dmy = 0u;
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    const int cp = CPL - 1 - k, cm = k;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      upx = fshr(upx, s.E[0][q][cp][1], 31);
      dpx = fshr(s.E[0][q][cp][0], dpx, 1);
      umx = fshr(umx, s.E[1][q][cm][1], 31);
      dmx = fshr(s.E[1][q][cm][0], dmx, 1);
    }
  }

  // ±y: maxima over columns c - 1 .. c + 1 of the row (in place), then the
  // shift by one row within the lane; the cross-wave bit follows the barrier
#pragma unroll
  for (int d = 2; d < 4; ++d) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      V4 left, right, prev;
#pragma unroll
      for (int q = 0; q < BITS_PLANES; ++q) {
        left.p[q] = q < B ? from_left<TORUS>(s.E[d][q][CPL - 1][w]) : 0u;  // lane i - 1, last column
        right.p[q] = q < B ? from_right<TORUS>(s.E[d][q][0][w]) : 0u;           // lane i + 1, first column
      }
      prev = left;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        V4 cur, nxt;
#pragma unroll
        for (int q = 0; q < BITS_PLANES; ++q) {
          cur.p[q] = s.E[d][q][c][w];
          nxt.p[q] = c + 1 < CPL ? s.E[d][q][c + 1][w] : right.p[q];
        }
        const V4 h = max3v<B>(prev, cur, nxt);
#pragma unroll
        for (int q = 0; q < B; ++q) s.E[d][q][c][w] = h.p[q];
        prev = cur;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const uint32_t h0 = s.E[d][q][c][0], h1 = s.E[d][q][c][1];
        if (d == 2) {  // +y reads the row below: word 1 now, word 0 after the exchange
          upy = fshr(upy, h1, 31);
          s.E[d][q][c][1] = fshr(h1, h0, 31);
        } else {  // -y reads the row above: word 0 now, word 1 after the exchange
          dmy = fshr(h0, dmy, 1);
          s.E[d][q][c][0] = fshr(h1, h0, 1);
        }
      }
  }

  XS[(v * 2 + 0) * 64 + lane] = make_uint4(upx, umx, upy, 0u);
  XS[(v * 2 + 1) * 64 + lane] = make_uint4(dpx, dmx, dmy, 0u);
  __syncthreads();
  // top row of the wave below, bottom row of the wave above (nothing beyond
  // the edges of a region that is not the whole torus: its halo absorbs that)
  const uint4 Bw = (!TORUS && v == 0) ? make_uint4(0u, 0u, 0u, 0u) : XS[(vdn * 2 + 0) * 64 + lane];
  const uint4 Aw = (!TORUS && v == CPL - 1) ? make_uint4(0u, 0u, 0u, 0u) : XS[(vup * 2 + 1) * 64 + lane];
  Carry cpx = {Bw.x << (32 - N), Aw.x >> (32 - N)};
  Carry cmx = {Bw.y << (32 - N), Aw.y >> (32 - N)};
  Carry cy = {Bw.z << (32 - N), Aw.z >> (32 - N)};

#pragma unroll
  for (int q = 0; q < B; ++q)
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      s.E[2][q][c][0] = fshr(s.E[2][q][c][0], cy.take_top(), 31);
      s.E[3][q][c][1] = fshr(cy.take_bot(), s.E[3][q][c][1], 1);
    }

  // +x: column c reads the vertical maxima of column c - 1
  {
    V4 r0, r1, h0, h1;
    constexpr int d = 0;
    bits_vmax<B, CPL>(s, d, CPL - 1, cpx, r0, r1);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      h0.p[q] = from_left<TORUS>(r0.p[q]);
      h1.p[q] = from_left<TORUS>(r1.p[q]);
    }
#pragma unroll
    for (int c = CPL - 1; c >= 1; --c) {
      bits_vmax<B, CPL>(s, d, c - 1, cpx, r0, r1);
#pragma unroll
      for (int q = 0; q < B; ++q) {
        s.E[d][q][c][0] = r0.p[q];
        s.E[d][q][c][1] = r1.p[q];
      }
      __builtin_amdgcn_sched_barrier(0);  // one column at a time: the state fills the register file
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      s.E[d][q][0][0] = h0.p[q];
      s.E[d][q][0][1] = h1.p[q];
    }
  }
  // -x: column c reads the vertical maxima of column c + 1
  {
    V4 r0, r1, h0, h1;
    constexpr int d = 1;
    bits_vmax<B, CPL>(s, d, 0, cmx, r0, r1);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      h0.p[q] = from_right<TORUS>(r0.p[q]);
      h1.p[q] = from_right<TORUS>(r1.p[q]);
    }
#pragma unroll
    for (int c = 0; c + 1 < CPL; ++c) {
      bits_vmax<B, CPL>(s, d, c + 1, cmx, r0, r1);
#pragma unroll
      for (int q = 0; q < B; ++q) {
        s.E[d][q][c][0] = r0.p[q];
        s.E[d][q][c][1] = r1.p[q];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      s.E[d][q][CPL - 1][0] = h0.p[q];
      s.E[d][q][CPL - 1][1] = h1.p[q];
    }
  }
}

// Moves of the anyons of one column word from the registers after the last
// sub-step of a step (see decide_site in band.h), every emission time below 2^B.
template <int B, int CPL>
__device__ __forceinline__ void bits_decide(const BitsLane<CPL> &s, int c, int w, uint32_t &px, uint32_t &mx,
                                            uint32_t &py, uint32_t &my) {
  uint32_t k[4];
  uint32_t m = s.E[0][B - 1][c][w] | s.E[1][B - 1][c][w] | s.E[2][B - 1][c][w] | s.E[3][B - 1][c][w];
  uint32_t nz = m;
#pragma unroll
  for (int d = 0; d < 4; ++d) k[d] = s.E[d][B - 1][c][w] | ~m;
#pragma unroll
  for (int q = B - 2; q >= 0; --q) {
    m = (s.E[0][q][c][w] & k[0]) | (s.E[1][q][c][w] & k[1]) | (s.E[2][q][c][w] & k[2]) | (s.E[3][q][c][w] & k[3]);
    nz |= m;
#pragma unroll
    for (int d = 0; d < 4; ++d) k[d] &= s.E[d][q][c][w] | ~m;
  }
  // k[d]: register d holds the site's largest emission time
  const uint32_t ok = s.S[c][w] & nz;
  const uint32_t sx = k[0], tx = k[1], sy = k[2], ty = k[3];
  py = ok & ty & ~sy;
  px = ok & ~ty & tx & ~sx;
  mx = ok & ~ty & ~tx & sx;
  my = ok & ~ty & ~tx & ~sx;
}

// Feedback of one decoder step: moves, OR'd link flips, syndrome update and
// the correction's winding bits (x-links leaving column L - 1: bit 2; y-links
// leaving row L - 1: bit 3).  Columns are decided one at a time, so that only
// one column's moves are live; the y-links across a wave boundary need one
// bit per column from each neighbour wave (MX: exchange area [wave][64]).
// Where the cuts of the winding parities lie in the workgroup's region: the
// x-links leaving column L - 1 are those of lane xlane's last column (-1:
// not in this region), counted on the rows of xrows; the y-links leaving row
// L - 1 are those above bit yb of word yw of wave yv (yv = -1: not in this
// region), counted on lanes [ylo, yhi).  On the whole torus: lane 63 on
// every row, and the top row of the top wave on every lane.
struct Cut {
  int xlane;
  uint32_t xrows[2];
  int yv, yw, yb, ylo, yhi;
};

template <int B, int CPL, bool TORUS>
__device__ __forceinline__ void bits_feedback(BitsLane<CPL> &s, uint2 *MX, int v, int vdn, int vup, int lane,
                                              uint32_t &wind, const Cut &cut) {
  // wind: the wave's winding bits (uniform)
  uint32_t upw = 0u, dnw = 0u;  // bit c: top-row +y move / bottom-row -y move of column c
  uint32_t ycut = 0u;           // parity of the cut's y-links flipped by this wave's own moves
  uint32_t pxl[2], mx0[2];      // previous column's +x moves; column 0's -x moves
  uint32_t xs[2];               // x-links of the last column
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    uint32_t px[2], mx[2], py[2], my[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) bits_decide<B, CPL>(s, c, w, px[w], mx[w], py[w], my[w]);
    // y-link above row y flips iff row y moves +y or row y + 1 moves -y; the
    // link above the top row also flips if the wave above moves -y there, the
    // link below the bottom row if the wave below moves +y there (after the
    // exchange).  Y of row y toggles rows y and y + 1.
    const uint32_t Y0 = py[0] | fshr(my[1], my[0], 1);
    const uint32_t Y1 = py[1] | (my[1] >> 1);
    s.S[c][0] ^= Y0 ^ (Y0 << 1);
    s.S[c][1] ^= Y1 ^ fshr(Y1, Y0, 31);
    upw |= (py[1] >> 31) << c;
    dnw |= (my[0] & 1u) << c;
    ycut ^= ((cut.yw ? Y1 : Y0) >> cut.yb) & 1u;
    if (c == 0) {
      mx0[0] = mx[0];
      mx0[1] = mx[1];
    } else {
#pragma unroll
      for (int w = 0; w < 2; ++w) {  // the x-link between columns c - 1 and c
        const uint32_t X = pxl[w] | mx[w];
        s.S[c - 1][w] ^= X;
        s.S[c][w] ^= X;
      }
    }
    pxl[0] = px[0];
    pxl[1] = px[1];
  }
#pragma unroll
  for (int w = 0; w < 2; ++w) {  // the x-link from the last column to lane i + 1's first
    xs[w] = pxl[w] | from_right<TORUS>(mx0[w]);
    s.S[CPL - 1][w] ^= xs[w];
    s.S[0][w] ^= from_left<TORUS>(xs[w]);
  }
  MX[v * 64 + lane] = make_uint2(upw, dnw);
  __syncthreads();
  const uint32_t pyb = (!TORUS && v == 0) ? 0u : MX[vdn * 64 + lane].x;        // wave below: its top row moves +y
  const uint32_t mya = (!TORUS && v == CPL - 1) ? 0u : MX[vup * 64 + lane].y;  // wave above: its bottom row moves -y
  // the link below the bottom row flips iff row 64v - 1 moves +y or row 64v
  // moves -y; the link above the top row iff the top row moves +y (applied
  // above) or row 64v + 64 moves -y
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    s.S[c][0] ^= ((pyb | dnw) >> c) & 1u;
    s.S[c][1] ^= (((mya & ~upw) >> c) & 1u) << 31;
  }
  uint32_t xb = 0u, yb = 0u;
  if (lane == cut.xlane) xb = (uint32_t)(__popc(xs[0] & cut.xrows[0]) + __popc(xs[1] & cut.xrows[1])) & 1u;
  if (v == cut.yv && lane >= cut.ylo && lane < cut.yhi) {
    // a link above a wave's top row also flips if the wave above moves -y into it
    const uint32_t above =
        (cut.yw == 1 && cut.yb == 31) ? (uint32_t)__popc(mya & ~upw & full_mask<CPL>()) : 0u;
    yb = (ycut ^ above) & 1u;
  }
  wind ^= wave_parity4((xb << 2) | (yb << 3));
}

// One decoder step (sub-steps t3 + 1 .. t3 + 3, then the feedback) with
// every emission time below 2^B, and below 2^B1 during its first sub-step
// (sub-step s needs the bit length of s: 1 at s = 1, 3 at s = 7).
template <int B, int CPL, int B1 = B, bool TORUS = true>
__device__ __forceinline__ void bits_step(BitsLane<CPL> &s, uint32_t t3, uint4 (*XS)[CPL * 2 * 64], uint2 *MX, int v,
                                       int vdn, int vup, int lane, uint32_t &wind, const Cut &cut) {
  uint32_t j = 1;
  if constexpr (B1 != B) {
    bits_substep<B1, CPL, TORUS>(s, t3 + 1u, XS[(t3 + 1u) & 1u], v, vdn, vup, lane);
    j = 2;
  }
#pragma unroll 1
  for (; j <= 3; ++j) bits_substep<B, CPL, TORUS>(s, t3 + j, XS[(t3 + j) & 1u], v, vdn, vup, lane);
  bits_feedback<B, CPL, TORUS>(s, MX, v, vdn, vup, lane, wind, cut);
}

// The emission times of word w (rows 4g_lo .. 4g_hi - 1 of the word) of a
// lane's four columns in the band layout: row y of the word (ybase + 4g + j,
// wrapped at L) goes to E[y P + q0] (columns 0, 1) and E[y P + q1] (columns
// 2, 3) as packed u16 pairs (e^{+x} | e^{-x} << 16, e^{+y} | e^{-y} << 16).
// Rows go four at a time: a plane's four bits of the group are spread to
// bit 0 of four bytes (a product with 2^0 + 2^7 + 2^14 + 2^21 places bit j at
// bit 8j, and the copies do not overlap; 24-bit products, one instruction),
// and the planes OR'd at bits q of those bytes, so byte j holds row 4g + j's
// emission time; one byte permutation then makes each 16-bit pair.
__device__ __forceinline__ void bits_store_rows(const BitsLane<4> &s, int w, int g_lo, int g_hi, int ybase, int L,
                                                int P, int q0, int q1, bool store, uint4 *E) {
  constexpr int CPL = 4;
#pragma unroll 1
  for (int g = g_lo; g < g_hi; ++g) {
    const uint32_t sh = opaque(4u * (uint32_t)g);
    uint32_t Z[4][CPL];
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        uint32_t z = 0u;
#pragma unroll
        for (int q = 0; q < BITS_PLANES; ++q)
          z |= q < 3 ? __umul24(__builtin_amdgcn_ubfe(s.E[d][q][c][w], sh, 4u), 0x00204081u << q) & (0x01010101u << q)
                     : (opaque(__umul24(__builtin_amdgcn_ubfe(s.E[d][q][c][w], sh, 4u), 0x00204081u)) & 0x01010101u)
                           << q;
        Z[d][c] = z;
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // byte 0: first operand's byte j, byte 2: second operand's byte j, bytes 1 and 3 zero
      const uint32_t sel = (uint32_t)j | 0x0C00u | ((uint32_t)(4 + j) << 16) | 0x0C000000u;
      uint32_t Pw[CPL], Qw[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        Pw[c] = __builtin_amdgcn_perm(Z[1][c], Z[0][c], sel);
        Qw[c] = __builtin_amdgcn_perm(Z[3][c], Z[2][c], sel);
      }
      int y = ybase + 4 * g + j;
      if (y >= L) y -= L;
      if (store) {
        E[(size_t)y * P + q0] = make_uint4(Pw[0], Qw[0], Pw[1], Qw[1]);
        E[(size_t)y * P + q1] = make_uint4(Pw[2], Qw[2], Pw[3], Qw[3]);
      }
    }
  }
}

// One workgroup per sample (DRAWN: the syndrome and error windings come from
// the noise kernel, in a.S_in and a.wind): noise, initial syndrome and windings, then up to
// a.k decoder steps, stopping after the first step that leaves no anyon.
// Writes the per-step anyon bits and the windings for k_finalize, and for a
// sample that still holds anyons its state in the band layout.
template <bool DRAWN, int CPL>
__global__ __launch_bounds__(CPL * 64) void k_bits(BitsArgs a) {
  constexpr int L = 64 * CPL, NW = CPL;
  __shared__ uint4 XS[2][NW * 2 * 64];
  __shared__ uint2 MX[NW * 64];
  __shared__ uint32_t red;
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int vdn = v == 0 ? NW - 1 : v - 1, vup = v == NW - 1 ? 0 : v + 1;
  const int64_t sample = a.order != nullptr ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
  if (a.zero_count != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.zero_count = 0;
  if (threadIdx.x == 0) red = 0u;

  BitsLane<CPL> s;
  uint32_t wind = 0u;
  if constexpr (DRAWN) {
    static_assert(CPL == 4, "drawn syndromes come from the L = 256 noise kernel");
    // the noise kernel's 16-row masks of column pairs: strips 4v + 2w and
    // 4v + 2w + 1 make word w; pairs 2i and 2i + 1 are this lane's columns
    const uint2 *Sp = a.S_in + (size_t)sample * (L / TILE_H) * (L / 2);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const size_t j = (size_t)(4 * v + 2 * w);
      const uint2 a0 = Sp[j * (L / 2) + 2 * lane], a1 = Sp[j * (L / 2) + 2 * lane + 1];
      const uint2 b0 = Sp[(j + 1) * (L / 2) + 2 * lane], b1 = Sp[(j + 1) * (L / 2) + 2 * lane + 1];
      s.S[0][w] = (a0.x & 0xFFFFu) | (b0.x << 16);
      s.S[1][w] = (a0.y & 0xFFFFu) | (b0.y << 16);
      s.S[2][w] = (a1.x & 0xFFFFu) | (b1.x << 16);
      s.S[3][w] = (a1.y & 0xFFFFu) | (b1.y << 16);
    }
  } else {
    const uint64_t seed = a.seeds[sample];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint64_t thr = a.p_arr ? device_threshold(a.p_arr[sample]) : a.thr;

    // noise: one Philox4x32-10 block (key = seed, counter = site index / 2)
    // per site pair, words 0 and 1 the x- and y-link of the even site, words
    // 2 and 3 those of the odd site; a link flips iff its word is below
    // thr.
    uint32_t ex[CPL][2], ey[CPL][2];
#pragma unroll
    for (int c = 0; c < CPL; ++c) ex[c][0] = ex[c][1] = ey[c][0] = ey[c][1] = 0u;
    // Rows from the top of each word down: a mask shifts left and takes the
    // new row's bit at bit 0 (m = 2 m + [word < thr] through the carry of
    // one v_addc), so row r ends at bit r.  thr = 2^32 (p = 1) flips every
    // link; below that the 32-bit comparison is exact.
    const uint32_t thr32 = thr > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)thr;
    if constexpr (CPL == 1) {
      // Lanes 2j and 2j + 1 (columns 2j, 2j + 1) share the blocks of site
      // pair j: the even lane draws the rows of word 0, the odd lane those
      // of word 1, each for both columns, and they swap the other column's half.
      const uint32_t par = (uint32_t)lane & 1u;
      uint32_t ax = 0u, ay = 0u, bx = 0u, by = 0u;  // columns 2j (a) and 2j + 1 (b), word par
#pragma unroll 4
      for (int r = 31; r >= 0; --r) {
        const uint32_t y = 32u * par + (uint32_t)r;
        const Words4 A = philox4x32_10(y * (L / 2) + ((uint32_t)lane >> 1), k0, k1);
        shift_in_below(ax, A.w0, thr32);
        shift_in_below(ay, A.w1, thr32);
        shift_in_below(bx, A.w2, thr32);
        shift_in_below(by, A.w3, thr32);
      }
      const uint32_t sax = swap_pair(ax), say = swap_pair(ay), sbx = swap_pair(bx), sby = swap_pair(by);
      ex[0][0] = par ? sbx : ax;
      ey[0][0] = par ? sby : ay;
      ex[0][1] = par ? bx : sax;
      ey[0][1] = par ? by : say;
    } else {
      // site pairs (CPL i + 2b, CPL i + 2b + 1), b < CPL / 2, of row y are
      // blocks y L/2 + (CPL/2) i + b
#pragma unroll
      for (int w = 0; w < 2; ++w) {
#pragma unroll 2
        for (int r = 31; r >= 0; --r) {
          const uint32_t y = (uint32_t)(64 * v + 32 * w + r);
          const uint32_t blk = y * (L / 2) + (uint32_t)(CPL / 2) * (uint32_t)lane;
#pragma unroll
          for (int b = 0; b < CPL / 2; ++b) {
            const Words4 A = philox4x32_10(blk + (uint32_t)b, k0, k1);
            shift_in_below(ex[2 * b][w], A.w0, thr32);
            shift_in_below(ey[2 * b][w], A.w1, thr32);
            shift_in_below(ex[2 * b + 1][w], A.w2, thr32);
            shift_in_below(ey[2 * b + 1][w], A.w3, thr32);
          }
        }
      }
    }
    if (thr > 0xFFFFFFFFull) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) ex[c][0] = ex[c][1] = ey[c][0] = ey[c][1] = ~0u;
    }
    uint32_t upw = 0u;
#pragma unroll
    for (int c = 0; c < CPL; ++c) upw |= (ey[c][1] >> 31) << c;
    MX[v * 64 + lane] = make_uint2(upw, 0u);
    __syncthreads();
    const uint32_t eyb = MX[vdn * 64 + lane].x;  // y-links above the top row of the wave below
    uint32_t wy = 0u;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const uint32_t xl0 = c > 0 ? ex[c - 1][0] : from_left<true>(ex[CPL - 1][0]);
      const uint32_t xl1 = c > 0 ? ex[c - 1][1] : from_left<true>(ex[CPL - 1][1]);
      s.S[c][0] = ex[c][0] ^ xl0 ^ ey[c][0] ^ ((ey[c][0] << 1) | ((eyb >> c) & 1u));
      s.S[c][1] = ex[c][1] ^ xl1 ^ ey[c][1] ^ fshr(ey[c][1], ey[c][0], 31);
      wy ^= ey[c][1] >> 31;
    }
    uint32_t wl = 0u;
    if (lane == 63) wl ^= (__popc(ex[CPL - 1][0]) + __popc(ex[CPL - 1][1])) & 1u;
    if (v == NW - 1) wl ^= wy << 1;
    wind = wave_parity4(wl);
  }
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int q = 0; q < BITS_PLANES; ++q)
#pragma unroll
      for (int c = 0; c < CPL; ++c) s.E[d][q][c][0] = s.E[d][q][c][1] = 0u;

  // anyons anywhere in the sample: a wave ballot, then (several waves) each
  // wave's flag through LDS -- every lane writes the same value -- and one
  // barrier (a block-wide OR intrinsic takes three)
  __shared__ uint32_t AF[NW];
  auto any_anyon = [&]() {
    uint32_t o = 0u;
#pragma unroll
    for (int c = 0; c < CPL; ++c) o |= s.S[c][0] | s.S[c][1];
    const bool wave_any = __ballot(o != 0u) != 0ull;
    if constexpr (NW == 1) {
      return wave_any;
    } else {
      AF[v] = wave_any ? 1u : 0u;
      __syncthreads();
      uint32_t r = 0u;
#pragma unroll
      for (int i = 0; i < NW; ++i) r |= AF[i];
      return __builtin_amdgcn_readfirstlane(r) != 0u;
    }
  };
  bool alive = any_anyon();
  uint32_t bits = alive ? 1u : 0u;
  int t = 0;
  // step t + 1 ends at sub-step 3 (t + 1): emission times below 4 in the
  // first step (below 2 in its first sub-step), below 8 in the second (and
  // the first sub-step of the third), below 16 up to the fifth, below 32 up
  // to the tenth
  const Cut cut = {63, {~0u, ~0u}, NW - 1, 1, 31, 0, 64};  // the whole torus
  auto after_step = [&]() {
    ++t;
    alive = any_anyon();
    if (alive) bits |= 1u << t;
  };
  if (alive && t < a.k) {
    bits_step<2, CPL, 1>(s, 0u, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  if (alive && t < a.k) {
    bits_step<3, CPL>(s, 3u, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  if (alive && t < a.k) {
    bits_step<4, CPL, 3>(s, 6u, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  while (alive && t < a.k && t < 5) {
    bits_step<4, CPL>(s, 3u * (uint32_t)t, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  while (alive && t < a.k) {
    bits_step<5, CPL>(s, 3u * (uint32_t)t, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }


  if (wind && lane_here() == 0) atomicXor(&red, wind);
  __syncthreads();
  // the sample index again (a scalar reload) rather than a value kept live
  // across the steps
  const int64_t smp = a.order != nullptr ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[opaque_s(blockIdx.x)])
                                         : (int64_t)blockIdx.x;
  if constexpr (CPL < 4) {
    // L = 64, 128: the decode's results when it ended inside these steps (no
    // anyon left, or T_max reached); else T_dec = -1 and the whole-lattice
    // kernel decodes the sample again from its seed
    (void)bits;
    const bool done = !alive || t >= a.T_max;
    if (threadIdx.x == 0) {
      if (done) {
        const uint32_t W = red;
        const uint32_t fail = ((W ^ (W >> 2)) & 3u) != 0u;
        const uint32_t timeout = alive ? 1u : 0u;
        a.T_dec[smp] = t;
        a.flags[smp] = (uint8_t)((fail | timeout) | (timeout << 1));
      } else {
        a.T_dec[smp] = -1;
      }
    }
    if (!done || a.syn == nullptr) return;
    // final syndrome, bit y L + x of the sample's row-major bitmap
    constexpr int NWORD = L * L / 32;
    uint32_t *out = a.syn + (size_t)smp * NWORD;
    if (!alive) {
      for (int i = threadIdx.x; i < NWORD; i += NW * 64) out[i] = 0u;
      return;
    }
    uint32_t *SW = reinterpret_cast<uint32_t *>(&XS[0][0]);  // free after the last step's barriers
    for (int i = threadIdx.x; i < NWORD; i += NW * 64) SW[i] = 0u;
    __syncthreads();
    for (int w = 0; w < 2; ++w)
      for (int c = 0; c < CPL; ++c)
        for (uint32_t m = s.S[c][w]; m != 0u; m &= m - 1u) {
          const uint32_t y = (uint32_t)(64 * v + 32 * w) + (uint32_t)__builtin_ctz(m);
          const uint32_t i = y * (uint32_t)L + (uint32_t)(CPL * lane + c);
          atomicOr(&SW[i >> 5], 1u << (i & 31u));
        }
    __syncthreads();
    for (int i = threadIdx.x; i < NWORD; i += NW * 64) out[i] = SW[i];
  } else {
    if (threadIdx.x == 0) {
      a.alive[smp] = bits;
      a.wind[smp] = DRAWN ? (a.wind[smp] ^ red) : red;  // the noise kernel left Wx(E), Wy(E)
    }
    if (!alive) return;
    // anyons left: the state in the band layout, emission times as packed u16
    // (P = e^{+x} | e^{-x} << 16, Q = e^{+y} | e^{-y} << 16) and 16-row syndrome masks
    constexpr size_t half_row = L / 2;
    const int ln = lane_here();
    uint4 *E = a.E + (size_t)smp * L * half_row;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      bits_store_rows(s, w, 0, 8, 64 * v + 32 * w, L, (int)half_row, 2 * ln, 2 * ln + 1, true, E);
      const size_t strip = (size_t)smp * (L / TILE_H) + (size_t)(4 * v + 2 * w);
      a.S[strip * half_row + 2 * ln] = make_uint2(s.S[0][w] & 0xFFFFu, s.S[1][w] & 0xFFFFu);
      a.S[strip * half_row + 2 * ln + 1] = make_uint2(s.S[2][w] & 0xFFFFu, s.S[3][w] & 0xFFFFu);
      a.S[(strip + 1) * half_row + 2 * ln] = make_uint2(s.S[0][w] >> 16, s.S[1][w] >> 16);
      a.S[(strip + 1) * half_row + 2 * ln + 1] = make_uint2(s.S[2][w] >> 16, s.S[3][w] >> 16);
    }
  }
}


// ---------------------------------------------------------------------------
// Tiled first pass for L > 256: each workgroup runs the same bit-sliced steps
// on a 256 x 256 region of one sample (four waves, four columns per lane),
// whose edges read nothing beyond it.  A decoder step moves information by
// at most 3 + 1 sites (three sub-steps of A^{(D)}, then the feedback), so
// after k steps the state is exact at least 4k sites inside the region's
// edges: the region keeps a halo of h = 4k rows and columns before its own
// part and at least as many after it.  The own parts (the L/4 groups of four
// rows or columns of a side split as evenly as possible over the tiles)
// cover the lattice once; every region runs all k steps (no early exit: its
// neighbours' anyons are not visible to it) and writes its own part of the
// state in the band layout -- the emission times row by row, the syndrome
// OR'd into 16-row masks that were cleared before (an own part need not
// start on a mask boundary).  Per-step anyon bits are OR'd and the
// correction windings XOR'd into the sample's words across tiles.

// Own part [o, o + w) of tile i of n along a side of L sites.
__device__ __forceinline__ void tile_owned(int L, int n, int i, int &o, int &w) {
  const int quads = L / 4, q = quads / n, r = quads % n;
  o = 4 * (i * q + (i < r ? i : r));
  w = 4 * (q + (i < r ? 1 : 0));
}

constexpr int BITS_TILE_MAX_STEPS = 6;  // halo 24; emission times up to 18 (5 planes)

struct BitsTileArgs {
  int L;
  int k;                 // decoder steps (<= BITS_TILE_MAX_STEPS and <= T_max)
  int halo;              // 4k
  int nt;                // tiles per side (nt x nt per sample)
  const int32_t *order;  // sample of grid row b: order[b] (nullptr: b)
  const uint2 *S_in;     // band layout [n][L/16][L/2] syndrome from the noise kernel (windings in wind)
  uint4 *E;              // band layout [n][L][L/2]: the state after the k steps
  uint2 *S;              // band layout [n][L/16][L/2], cleared before
  uint32_t *alive;       // per sample (zeroed before): bit j anyons after step j, OR over tiles
  uint32_t *wind;        // per sample: error windings in, correction windings XOR'd over tiles
  int *zero_count;       // survivor counter of the following compaction (cleared here)
};

__global__ __launch_bounds__(256) void k_bits_tile(BitsTileArgs a) {
  constexpr int CPL = 4, NW = 4;
  __shared__ uint4 XS[2][NW * 2 * 64];
  __shared__ uint2 MX[NW * 64];
  __shared__ uint32_t red;
  __shared__ uint32_t AF[NW];
  const int L = a.L, P = L / 2, NS = L / TILE_H, h = a.halo;
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int vdn = v == 0 ? NW - 1 : v - 1, vup = v == NW - 1 ? 0 : v + 1;
  const int64_t smp = a.order != nullptr ? (int64_t)a.order[blockIdx.y] : (int64_t)blockIdx.y;
  int ox, owx, oy, owy;
  tile_owned(L, a.nt, (int)(blockIdx.x % (unsigned)a.nt), ox, owx);
  tile_owned(L, a.nt, (int)(blockIdx.x / (unsigned)a.nt), oy, owy);
  // (indices below twice their range wrap by one subtraction)
  auto wrap = [](int i, int n) { return i >= n ? i - n : i; };
  const int X0 = wrap(ox - h + L, L), Y0 = wrap(oy - h + L, L);  // region origin (multiples of 4)
  if (a.zero_count != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.zero_count = 0;
  if (threadIdx.x == 0) red = 0u;

  // own part: rows [h, h + owy) and lanes [h/4, (h + owx)/4) of the region
  uint32_t own_rows[2];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int r0 = 64 * v + 32 * w;
    const int lo = min(max(h - r0, 0), 32), hi = min(max(h + owy - r0, 0), 32);
    own_rows[w] = (hi > lo ? (hi - lo == 32 ? ~0u : ((1u << (hi - lo)) - 1u)) : 0u) << (lo & 31);
  }
  const int own_lo = h / 4, own_hi = (h + owx) / 4;  // own lanes
  const uint64_t own_mask = (own_hi == 64 ? ~0ull : ((1ull << own_hi) - 1ull)) & ~((1ull << own_lo) - 1ull);

  // the noise kernel's 16-row masks: word w starts at lattice row
  // Y0 + 64v + 32w, `off` rows into a mask, and spans that mask and the next
  // two; column pairs (X0 + 4i)/2 and the next are this lane's columns
  BitsLane<CPL> s;
  const int p0 = wrap(X0 / 2 + 2 * lane, P), p1 = wrap(p0 + 1, P);
  {
    const uint2 *Sp = a.S_in + (size_t)smp * NS * P;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int R = wrap(Y0 + 64 * v + 32 * w, L), off = R % TILE_H;
      const int j0 = R / TILE_H, j1 = wrap(j0 + 1, NS), j2 = wrap(j0 + 2, NS);
      uint64_t m[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int j = i == 0 ? j0 : (i == 1 ? j1 : j2);
        const uint2 u0 = Sp[(size_t)j * P + p0], u1 = Sp[(size_t)j * P + p1];
        m[0] |= (uint64_t)(u0.x & 0xFFFFu) << (16 * i);
        m[1] |= (uint64_t)(u0.y & 0xFFFFu) << (16 * i);
        m[2] |= (uint64_t)(u1.x & 0xFFFFu) << (16 * i);
        m[3] |= (uint64_t)(u1.y & 0xFFFFu) << (16 * i);
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) s.S[c][w] = (uint32_t)(m[c] >> off);
    }
  }
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int q = 0; q < BITS_PLANES; ++q)
#pragma unroll
      for (int c = 0; c < CPL; ++c) s.E[d][q][c][0] = s.E[d][q][c][1] = 0u;

  auto own_anyon = [&]() {
    uint32_t o = 0u;
#pragma unroll
    for (int c = 0; c < CPL; ++c) o |= (s.S[c][0] & own_rows[0]) | (s.S[c][1] & own_rows[1]);
    return (__ballot(o != 0u) & own_mask) != 0ull;  // uniform in the wave
  };
  // anyons in the whole own part: each wave's flag through LDS (every lane
  // writes the same value), one barrier
  auto group_any = [&]() {
    AF[v] = own_anyon() ? 1u : 0u;
    __syncthreads();
    uint32_t o = 0u;
#pragma unroll
    for (int i = 0; i < NW; ++i) o |= AF[i];
    return __builtin_amdgcn_readfirstlane(o) != 0u;
  };
  // the cuts of the winding parities, where this tile owns them
  Cut cut;
  cut.xlane = ox + owx == L ? (h + owx) / 4 - 1 : -1;
  cut.xrows[0] = own_rows[0];
  cut.xrows[1] = own_rows[1];
  const int ry = h + owy - 1;  // region row of lattice row L - 1 (if owned)
  cut.yv = oy + owy == L ? ry / 64 : -1;
  cut.yw = (ry % 64) / 32;
  cut.yb = ry % 32;
  cut.ylo = own_lo;
  cut.yhi = own_hi;

  uint32_t wind = 0u;
  uint32_t bits = group_any() ? 1u : 0u;
  int t = 0;
  auto after_step = [&]() {
    ++t;
    if (group_any()) bits |= 1u << t;
  };
  if (t < a.k) {
    bits_step<2, CPL, 1, false>(s, 0u, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  if (t < a.k) {
    bits_step<3, CPL, 3, false>(s, 3u, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  if (t < a.k) {
    bits_step<4, CPL, 3, false>(s, 6u, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  while (t < a.k && t < 5) {
    bits_step<4, CPL, 4, false>(s, 3u * (uint32_t)t, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }
  if (t < a.k) {
    bits_step<5, CPL, 5, false>(s, 15u, XS, MX, v, vdn, vup, lane, wind, cut);
    after_step();
  }

  if (wind && lane_here() == 0) atomicXor(&red, wind);
  __syncthreads();
  const int64_t sm2 = a.order != nullptr ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[opaque_s(blockIdx.y)])
                                         : (int64_t)blockIdx.y;
  if (threadIdx.x == 0) {
    if (red) atomicXor(&a.wind[sm2], red);
    atomicOr(&a.alive[sm2], bits);
  }
  // own part of the state in the band layout (own rows come in groups of four)
  const int ln = lane_here();
  const bool own = ln >= own_lo && ln < own_hi;
  const int q0 = wrap(X0 / 2 + 2 * ln, P), q1 = wrap(q0 + 1, P);
  uint4 *E = a.E + (size_t)sm2 * L * P;
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int r0 = 64 * v + 32 * w;
    const int g_lo = min(max(h - r0, 0), 32) / 4, g_hi = min(max(h + owy - r0, 0), 32) / 4;
    bits_store_rows(s, w, g_lo, g_hi, wrap(Y0 + r0, L), L, P, q0, q1, own, E);
    // syndrome: the word's own rows, shifted to their place in the masks
    // (anyons only: the masks were cleared)
    const int R = wrap(Y0 + r0, L), off = R % TILE_H, j0 = R / TILE_H;
    uint2 *Sd = a.S + (size_t)sm2 * NS * P;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const uint64_t m = own ? (uint64_t)(s.S[c][w] & own_rows[w]) << off : 0ull;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const uint32_t part = (uint32_t)(m >> (16 * i)) & 0xFFFFu;
        if (part != 0u) {
          const int j = wrap(j0 + i, NS);
          uint32_t *dst = reinterpret_cast<uint32_t *>(&Sd[(size_t)j * P + (c < 2 ? q0 : q1)]) + (c & 1);
          atomicOr(dst, part);
        }
      }
    }
  }
}

}  // namespace mpd
