// torus.h -- whole-lattice band engine with one column per lane (gfx950).
//
// For an L = 64 torus a wave holds all 64 columns of a 16-row strip, one
// column per lane, so the periodic wrap in x is a wave-wide DPP rotation
// (band.h's from_left<true> / from_right<true>) and no halo exists; rows of
// the strip are the lane's own registers and only the strip's first and last
// rows go through LDS.  Register layout per site as in engine.h: P =
// e^{+x} | e^{-x} << 16, Q = e^{+y} | e^{-y} << 16 (emission times); the
// syndrome bits of a lane are a 16-bit mask (bit h = row h of the strip).
// The two-column form for L = 128 is band.h's band_substep / band_feedback
// with ROT.
#pragma once

#include "band.h"

namespace mpd {

// Anyon sites of the rows flagged in `rows` (wave-uniform) publish "emits
// now" (the sub-step time ss in both halves).
template <int H>
__device__ __forceinline__ void col_fold(uint32_t (&P)[H], uint32_t (&Q)[H], uint32_t s, uint32_t ss,
                                         uint32_t rows) {
  asm volatile("" : "+v"(s));
#pragma unroll
  for (int h = 0; h < H; ++h) {
    if (!((rows >> h) & 1u)) continue;
    const uint32_t m = (uint32_t)((int32_t)(s << (31 - h)) >> 31);
    P[h] = (ss & m) | (P[h] & ~m);
    Q[h] = (ss & m) | (Q[h] & ~m);
  }
}

// Maximum of Q over the columns c - 1, c, c + 1 of one row (periodic).
__device__ __forceinline__ uint32_t col_hmax(uint32_t q) {
  return pmax(pmax(q, from_left<true>(q)), from_right<true>(q));
}

// One application of A^{(D)} to a one-column strip (registers folded on
// entry, new emission times on exit).  BND: this sub-step's LDS slot,
// [wave][2][64] of (P, Q) for the strip's first and last rows; wdn / wup the
// waves below and above (periodic).  With DECIDE the moves of the anyons in
// the flagged rows are decided from the new values.
template <int H, bool DECIDE>
__device__ __forceinline__ void col_substep(uint32_t (&P)[H], uint32_t (&Q)[H], uint32_t s, uint2 *BND, int w,
                                            int wdn, int wup, int lane, uint32_t rows, uint32_t ethr, Moves &mv) {
  BND[(w * 2 + 0) * 64 + lane] = make_uint2(P[0], Q[0]);
  BND[(w * 2 + 1) * 64 + lane] = make_uint2(P[H - 1], Q[H - 1]);
  __syncthreads();
  const uint2 dn = BND[(wdn * 2 + 1) * 64 + lane];  // row just below the strip
  uint32_t hqm = col_hmax(dn.y), hqc = col_hmax(Q[0]);
  uint32_t pm = pmax(dn.x, P[0]);  // vertical pair maximum (h - 1, h)
#pragma unroll
  for (int h = 0; h < H; ++h) {
    constexpr int last = H - 1;
    const int hn = h < last ? h + 1 : last;
    uint2 up = make_uint2(0u, 0u);
    if (h == last) up = BND[(wup * 2 + 0) * 64 + lane];  // row just above the strip
    const uint32_t pnx = h < last ? P[hn] : up.x;
    const uint32_t qnx = h < last ? Q[hn] : up.y;
    const uint32_t hqn = col_hmax(qnx);
    const uint32_t pn = pmax(P[h], pnx);
    const uint32_t vm = pmax(pm, pn);  // vertical maximum over rows h - 1 .. h + 1
    pm = pn;
    P[h] = lohi(from_left<true>(vm), from_right<true>(vm));  // +x from column c - 1, -x from c + 1
    Q[h] = lohi(hqm, hqn);                                    // +y from the row below, -y from above
    hqm = hqc;
    hqc = hqn;
    if (DECIDE && ((rows >> h) & 1u)) decide_site(P[h], Q[h], (s >> h) & 1u, 1u << h, ethr, mv);
  }
}

// Feedback of a one-column strip: OR of both endpoints' moves per link (eq.
// (ddfeedback)), new syndrome mask.  MB: LDS [wave][64] for the y-moves at
// strip edges.  xo receives the flipped x-links to the right of the column,
// yo the flipped y-links above each row.
template <int H>
__device__ __forceinline__ uint32_t col_feedback(uint32_t s, const Moves &mv, uint2 *MB, int w, int wdn, int wup,
                                                 int lane, uint32_t &xo, uint32_t &yo) {
  static_assert(H <= 16, "move masks hold 16 rows");
  MB[w * 64 + lane] = make_uint2(mv.py, mv.my);
  __syncthreads();
  const uint32_t upmy = MB[wup * 64 + lane].y;  // wave above: bit 0 = its first row moves -y
  const uint32_t dnpy = MB[wdn * 64 + lane].x;  // wave below: bit H-1 = its last row moves +y
  constexpr uint32_t F = full_mask<H>();
  xo = (mv.px | from_right<true>(mv.mx)) & F;  // column c moves +x, or c + 1 moves -x
  const uint32_t xl = from_left<true>(xo);     // the link from column c - 1
  yo = (mv.py | (mv.my >> 1) | ((upmy & 1u) << (H - 1))) & F;
  const uint32_t yd = ((mv.py << 1) | ((dnpy >> (H - 1)) & 1u) | mv.my) & F;
  return (s ^ xo ^ xl ^ yo ^ yd) & F;
}

}  // namespace mpd
