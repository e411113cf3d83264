// band.h -- register-resident band engine for large lattices (gfx950).
//
// A workgroup of NW waves holds a region of 128 columns x (NW * H) rows of
// one sample.  Lane i of every wave owns the two adjacent region columns 2i
// and 2i+1 over the wave's H rows, with the packed emission-time registers
// of engine.h (P = e^{+x} | e^{-x} << 16, Q = e^{+y} | e^{-y} << 16) in
// VGPRs.  Horizontal neighbours are read with wave-wide DPP lane shifts
// (wave_shr / wave_shl), vertical ones from the lane's own registers; only
// the rows at wave boundaries go through LDS.  Columns beyond the region
// edge read the edge lane's own value: the halo absorbs that.
//
// Syndrome bits of a lane: s0 bit h = column 2i, row h; s1 bit h = column
// 2i+1, row h (H <= 32).
#pragma once

#include "engine.h"

namespace mpd {

// Wave-wide DPP controls (GFX9).  Lanes whose source lies outside the wave
// read 0 (bound_ctrl), which lets the compiler fold the shift into the
// consuming instruction; those edge lanes only feed the halo.
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane i <- lane i+1
constexpr int DPP_WAVE_ROL1 = 0x134;  // lane i <- lane i+1 mod 64
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane i <- lane i-1
constexpr int DPP_WAVE_ROR1 = 0x13C;  // lane i <- lane i-1 mod 64

// Neighbour lanes' values.  ROT: the wave is periodic (a region that spans
// the lattice's width with 64 lanes, the torus wrap in x); otherwise the
// edge lanes read 0 and only feed a halo.
template <bool ROT = false>
__device__ __forceinline__ uint32_t from_left(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ROT ? DPP_WAVE_ROR1 : DPP_WAVE_SHR1, 0xF, 0xF, !ROT);
}
template <bool ROT = false>
__device__ __forceinline__ uint32_t from_right(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ROT ? DPP_WAVE_ROL1 : DPP_WAVE_SHL1, 0xF, 0xF, !ROT);
}

// low 16 bits from a, high 16 bits from b
__device__ __forceinline__ uint32_t lohi(uint32_t a, uint32_t b) {
  return (a & 0xFFFFu) | (b & 0xFFFF0000u);
}

template <int H>
struct BandLane {
  uint32_t P0[H], Q0[H], P1[H], Q1[H];
  uint32_t s0, s1;
};

// Moves of a strip's anyons: bit h + 16c of px = the anyon in column c
// (0/1), row h moves +x (likewise -x, +y, -y).  H <= 16.
struct Moves {
  uint32_t px, mx, py, my;
};

// Move decision of one site from its registers (see engine.h): the largest
// emission time wins (smallest message), ties in the order -y, -x, +x, +y,
// and no move if the opposite register on that axis ties.  Registers below
// `ethr` (live_threshold) hold no live message.  Sets bit `bit` of the mask
// of the chosen move; `anyon` gates it.
__device__ __forceinline__ void decide_site(uint32_t P, uint32_t Q, bool anyon, uint32_t bit, uint32_t ethr,
                                            Moves &mv) {
  // The row bit lives in an SGPR set where it is used: as a literal it would
  // be materialised in a VGPR of its own per row and hoisted out of every loop.
  asm volatile("" : "+s"(bit));
  const uint32_t T = pmax(P, Q);  // (max(+x, +y), max(-x, -y))
  const uint16_t M = max((uint16_t)T, (uint16_t)(T >> 16));
  const bool sx = (uint16_t)P == M, tx = (uint16_t)(P >> 16) == M;
  const bool sy = (uint16_t)Q == M, ty = (uint16_t)(Q >> 16) == M;
  const bool ok = anyon && (uint32_t)M >= ethr;
  const bool go_py = ok && ty && !sy;
  const bool go_px = ok && !ty && tx && !sx;
  const bool go_mx = ok && !ty && !tx && sx;
  const bool go_my = ok && !ty && !tx && !sx;
  mv.py |= go_py ? bit : 0u;
  mv.px |= go_px ? bit : 0u;
  mv.mx |= go_mx ? bit : 0u;
  mv.my |= go_my ? bit : 0u;
}

// Rows of the wave that hold an anyon in any lane (wave-uniform).
template <int H>
__device__ __forceinline__ uint32_t wave_rows(uint32_t s0, uint32_t s1) {
  uint32_t rows = 0u;
  const uint32_t both = s0 | s1;
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (__builtin_amdgcn_ballot_w64(((both >> h) & 1u) != 0u)) rows |= 1u << h;
  return rows;
}

// Anyon sites publish "emits now": their registers read as the sub-step time.
// Only rows flagged in `rows` (wave-uniform: rows holding an anyon in some
// lane) are touched -- after the first decoder step most rows hold none.
template <int H>
__device__ __forceinline__ void band_fold(BandLane<H> &b, uint32_t ss, uint32_t rows) {
  // The masks do not change between the sub-steps of a step; keep the
  // compiler from hoisting 2*H lane masks out of the sub-step loop.
  asm volatile("" : "+v"(b.s0), "+v"(b.s1));
#pragma unroll
  for (int h = 0; h < H; ++h) {
    if (!((rows >> h) & 1u)) continue;
    // all-ones where row h holds an anyon (sign extension of bit h)
    const uint32_t m0 = (uint32_t)((int32_t)(b.s0 << (31 - h)) >> 31);
    const uint32_t m1 = (uint32_t)((int32_t)(b.s1 << (31 - h)) >> 31);
    b.P0[h] = (ss & m0) | (b.P0[h] & ~m0);
    b.Q0[h] = (ss & m0) | (b.Q0[h] & ~m0);
    b.P1[h] = (ss & m1) | (b.P1[h] & ~m1);
    b.Q1[h] = (ss & m1) | (b.Q1[h] & ~m1);
  }
}

// Open lattice: before every update, lanes outside the lattice hold
// nothing, and a rough-boundary column (bL: the lane's first column is
// x = 0, bR: its second is x = L-1) reads as "emits now" in P, so that the
// x-registers of its bulk neighbour receive a message of value 1, and as
// nothing in Q.
template <int H>
__device__ __forceinline__ void band_boundary_fold(BandLane<H> &b, uint32_t ss, bool outside, bool bL, bool bR) {
#pragma unroll
  for (int h = 0; h < H; ++h) {
    if (outside) b.P0[h] = b.Q0[h] = b.P1[h] = b.Q1[h] = 0u;
    if (bL) {
      b.P0[h] = ss;
      b.Q0[h] = 0u;
    }
    if (bR) {
      b.P1[h] = ss;
      b.Q1[h] = 0u;
    }
  }
}

// One application of A^{(D)} to the band (registers hold folded values on
// entry and the new emission times on exit).  BND is this sub-step's LDS
// slot for boundary rows: [wave][2][64] of (P0, Q0, P1, Q1).  With DECIDE
// (last sub-step of a decoder step) the moves of the anyons in the rows
// flagged in `rows` are decided from the new values as each row completes.
template <int H, bool DECIDE, bool ROT = false>
__device__ __forceinline__ void band_substep(BandLane<H> &b, uint4 *BND, int w, int wdn, int wup, int lane,
                                             uint32_t rows, uint32_t ethr, Moves &mv) {
  BND[(w * 2 + 0) * 64 + lane] = make_uint4(b.P0[0], b.Q0[0], b.P1[0], b.Q1[0]);
  BND[(w * 2 + 1) * 64 + lane] = make_uint4(b.P0[H - 1], b.Q0[H - 1], b.P1[H - 1], b.Q1[H - 1]);
  __syncthreads();
  const uint4 dn = BND[(wdn * 2 + 1) * 64 + lane];  // row just below the strip

  // hq0/hq1: max of Q over columns (2i-1, 2i, 2i+1) / (2i, 2i+1, 2i+2) of a
  // row; suffix m = row below the current one, c = current, n = above.
  uint32_t hq0m, hq1m, hq0c, hq1c;
  {
    const uint32_t t = pmax(dn.y, dn.w);
    hq0m = pmax(t, from_left<ROT>(dn.w));
    hq1m = pmax(t, from_right<ROT>(dn.y));
    const uint32_t t2 = pmax(b.Q0[0], b.Q1[0]);
    hq0c = pmax(t2, from_left<ROT>(b.Q1[0]));
    hq1c = pmax(t2, from_right<ROT>(b.Q0[0]));
  }
  // vertical max of P over rows h-1..h+1 as max of the pair maxima
  // (h-1, h) and (h, h+1): the old P of row h is then dead before its new
  // value is written, so the update runs in place.
  uint32_t pm0 = pmax(dn.x, b.P0[0]), pm1 = pmax(dn.z, b.P1[0]);
#pragma unroll
  for (int h = 0; h < H; ++h) {
    constexpr int last = H - 1;
    const int hn = h < last ? h + 1 : last;  // in range for every h; unused at h = last
    uint4 up = make_uint4(0u, 0u, 0u, 0u);   // row just above the strip, read when needed
    if (h == last) up = BND[(wup * 2 + 0) * 64 + lane];
    const uint32_t p0n = h < last ? b.P0[hn] : up.x;
    const uint32_t p1n = h < last ? b.P1[hn] : up.z;
    const uint32_t q0n = h < last ? b.Q0[hn] : up.y;
    const uint32_t q1n = h < last ? b.Q1[hn] : up.w;
    const uint32_t tn = pmax(q0n, q1n);
    const uint32_t hq0n = pmax(tn, from_left<ROT>(q1n));
    const uint32_t hq1n = pmax(tn, from_right<ROT>(q0n));
    const uint32_t pn0 = pmax(b.P0[h], p0n), pn1 = pmax(b.P1[h], p1n);
    const uint32_t vm0 = pmax(pm0, pn0);  // vertical max, column 2i
    const uint32_t vm1 = pmax(pm1, pn1);  // vertical max, column 2i+1
    pm0 = pn0;
    pm1 = pn1;
    b.P0[h] = lohi(from_left<ROT>(vm1), vm1);   // +x from column 2i-1, -x from 2i+1
    b.P1[h] = lohi(vm0, from_right<ROT>(vm0));  // +x from column 2i, -x from 2i+2
    b.Q0[h] = lohi(hq0m, hq0n);            // +y from the row below, -y from above
    b.Q1[h] = lohi(hq1m, hq1n);
    hq0m = hq0c;
    hq1m = hq1c;
    hq0c = hq0n;
    hq1c = hq1n;
    if (DECIDE && ((rows >> h) & 1u)) {  // wave-uniform: rows holding an anyon
      decide_site(b.P0[h], b.Q0[h], (b.s0 >> h) & 1u, 1u << h, ethr, mv);
      decide_site(b.P1[h], b.Q1[h], (b.s1 >> h) & 1u, 1u << (16 + h), ethr, mv);
    }
  }
}

// Random moves of a random-move step t (limited-memory variant, see
// engine.h) for the anyons in the rows flagged in `rows`: the lane's two
// columns gx, gx + 1 (gx even) of row gy + h are the sites of generator
// pair ((gy + h) L + gx) / 2.
template <int H>
__device__ __forceinline__ void band_random_moves(const BandLane<H> &b, uint32_t rows, int gx, int gy, int L,
                                                  uint32_t t, uint32_t k0, uint32_t k1, Moves &mv) {
  for (int h = 0; h < H; ++h) {
    if (!((rows >> h) & 1u)) continue;
    const uint2 d = random_dirs((uint32_t)(((gy + h) * L + gx) >> 1), t, k0, k1);
    const uint32_t b0 = ((b.s0 >> h) & 1u) << h, b1 = ((b.s1 >> h) & 1u) << (16 + h);
    mv.px |= (d.x == 0u ? b0 : 0u) | (d.y == 0u ? b1 : 0u);
    mv.mx |= (d.x == 1u ? b0 : 0u) | (d.y == 1u ? b1 : 0u);
    mv.py |= (d.x == 2u ? b0 : 0u) | (d.y == 2u ? b1 : 0u);
    mv.my |= (d.x == 3u ? b0 : 0u) | (d.y == 3u ? b1 : 0u);
  }
}

// Feedback for the band: link flips from the moves (OR of both endpoints,
// eq. (ddfeedback)) and the syndrome update.  MB is an LDS array [wave][64]
// used to pass the y-moves across wave boundaries.  xo[c] receives the
// flipped x-links to the right of column c, yo[c] the flipped y-links above
// each row of column c.
template <int H, bool ROT = false>
__device__ __forceinline__ void band_feedback(BandLane<H> &b, const Moves &mv, uint2 *MB, int w, int wdn,
                                              int wup, int lane, uint32_t (&xo)[2], uint32_t (&yo)[2]) {
  static_assert(H <= 16, "move masks hold 16 rows per column");
  MB[w * 64 + lane] = make_uint2(mv.py, mv.my);
  __syncthreads();
  const uint32_t upmy = MB[wup * 64 + lane].y;  // wave above: bit 16c = its first row moves -y
  const uint32_t dnpy = MB[wdn * 64 + lane].x;  // wave below: bit 16c+H-1 = its last row moves +y
  constexpr uint32_t F = full_mask<H>();
  // x-links: column 2i -> 2i+1 and column 2i+1 -> 2i+2 (next lane's column 2i)
  xo[0] = (mv.px | (mv.mx >> 16)) & F;
  xo[1] = ((mv.px >> 16) | from_right<ROT>(mv.mx)) & F;
  const uint32_t xl0 = from_left<ROT>(xo[1]), xl1 = xo[0];
  {
    const uint32_t py = mv.py & F, my = mv.my & F;
    const uint32_t yd = ((py << 1) | ((dnpy >> (H - 1)) & 1u) | my) & F;
    yo[0] = (py | (my >> 1) | ((upmy & 1u) << (H - 1))) & F;
    b.s0 = (b.s0 ^ xo[0] ^ xl0 ^ yo[0] ^ yd) & F;
  }
  {
    const uint32_t py = (mv.py >> 16) & F, my = (mv.my >> 16) & F;
    const uint32_t yd = ((py << 1) | ((dnpy >> (16 + H - 1)) & 1u) | my) & F;
    yo[1] = (py | (my >> 1) | (((upmy >> 16) & 1u) << (H - 1))) & F;
    b.s1 = (b.s1 ^ xo[1] ^ xl1 ^ yo[1] ^ yd) & F;
  }
}

}  // namespace mpd
