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

// Wave-wide DPP controls (GFX9): a lane whose source lies outside the wave
// keeps its own value.
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane i <- lane i+1
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane i <- lane i-1

__device__ __forceinline__ uint32_t from_left(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_WAVE_SHR1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_right(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_WAVE_SHL1, 0xF, 0xF, false);
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

// Moves of a strip's anyons: bit h of px[c] = the anyon in column c, row h
// moves +x (likewise -x, +y, -y).
struct Moves {
  uint32_t px[2], mx[2], py[2], my[2];
};

// Move decision of one site from its registers, branch-free (see engine.h).
// Returns the moves as bits (bit 0 +x, bit 1 -x, bit 2 +y, bit 3 -y): the
// largest emission time wins (smallest message), ties in the order -y, -x,
// +x, +y, and no move if the opposite register on that axis ties.  `anyon`
// is 0 or 1; non-anyon sites return 0.
__device__ __forceinline__ uint32_t decide_site(uint32_t P, uint32_t Q, uint32_t anyon) {
  const uint32_t vpx = P & 0xFFFFu, vmx = P >> 16, vpy = Q & 0xFFFFu, vmy = Q >> 16;
  const uint32_t M = max(max(vpx, vmx), max(vpy, vmy));
  const uint32_t ty = vmy == M, tx = vmx == M, sx = vpx == M, sy = vpy == M;
  const uint32_t go_py = ty & (sy ^ 1u);
  const uint32_t go_px = (ty ^ 1u) & tx & (sx ^ 1u);
  const uint32_t go_mx = (ty ^ 1u) & (tx ^ 1u) & sx;
  const uint32_t go_my = (ty ^ 1u) & (tx ^ 1u) & (sx ^ 1u);
  const uint32_t code = go_px | (go_mx << 1) | (go_py << 2) | (go_my << 3);
  return code & (0u - (anyon & (uint32_t)(M != 0u)));
}

__device__ __forceinline__ void add_moves(Moves &mv, int c, int h, uint32_t code) {
  mv.px[c] |= (code & 1u) << h;
  mv.mx[c] |= ((code >> 1) & 1u) << h;
  mv.py[c] |= ((code >> 2) & 1u) << h;
  mv.my[c] |= ((code >> 3) & 1u) << h;
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
// Branch-free per row; the caller skips it for waves without anyons.
template <int H>
__device__ __forceinline__ void band_fold(BandLane<H> &b, uint32_t ss) {
  // The masks do not change between the sub-steps of a step; keep the
  // compiler from hoisting 2*H lane masks out of the sub-step loop.
  asm volatile("" : "+v"(b.s0), "+v"(b.s1));
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const bool a0 = (b.s0 >> h) & 1u, a1 = (b.s1 >> h) & 1u;
    b.P0[h] = a0 ? ss : b.P0[h];
    b.Q0[h] = a0 ? ss : b.Q0[h];
    b.P1[h] = a1 ? ss : b.P1[h];
    b.Q1[h] = a1 ? ss : b.Q1[h];
  }
}

// One application of A^{(D)} to the band (registers hold folded values on
// entry and the new emission times on exit).  BND is this sub-step's LDS
// slot for boundary rows: [wave][2][64] of (P0, Q0, P1, Q1).  With DECIDE
// (last sub-step of a decoder step) the moves of the anyons in the rows
// flagged in `rows` are decided from the new values as each row completes.
template <int H, bool DECIDE>
__device__ __forceinline__ void band_substep(BandLane<H> &b, uint4 *BND, int w, int wdn, int wup, int lane,
                                             uint32_t rows, Moves &mv) {
  BND[(w * 2 + 0) * 64 + lane] = make_uint4(b.P0[0], b.Q0[0], b.P1[0], b.Q1[0]);
  BND[(w * 2 + 1) * 64 + lane] = make_uint4(b.P0[H - 1], b.Q0[H - 1], b.P1[H - 1], b.Q1[H - 1]);
  __syncthreads();
  const uint4 dn = BND[(wdn * 2 + 1) * 64 + lane];  // row just below the strip

  // hq0/hq1: max of Q over columns (2i-1, 2i, 2i+1) / (2i, 2i+1, 2i+2) of a
  // row; suffix m = row below the current one, c = current, n = above.
  uint32_t hq0m, hq1m, hq0c, hq1c;
  {
    const uint32_t t = pmax(dn.y, dn.w);
    hq0m = pmax(t, from_left(dn.w));
    hq1m = pmax(t, from_right(dn.y));
    const uint32_t t2 = pmax(b.Q0[0], b.Q1[0]);
    hq0c = pmax(t2, from_left(b.Q1[0]));
    hq1c = pmax(t2, from_right(b.Q0[0]));
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
    const uint32_t hq0n = pmax(tn, from_left(q1n));
    const uint32_t hq1n = pmax(tn, from_right(q0n));
    const uint32_t pn0 = pmax(b.P0[h], p0n), pn1 = pmax(b.P1[h], p1n);
    const uint32_t vm0 = pmax(pm0, pn0);  // vertical max, column 2i
    const uint32_t vm1 = pmax(pm1, pn1);  // vertical max, column 2i+1
    pm0 = pn0;
    pm1 = pn1;
    b.P0[h] = lohi(from_left(vm1), vm1);   // +x from column 2i-1, -x from 2i+1
    b.P1[h] = lohi(vm0, from_right(vm0));  // +x from column 2i, -x from 2i+2
    b.Q0[h] = lohi(hq0m, hq0n);            // +y from the row below, -y from above
    b.Q1[h] = lohi(hq1m, hq1n);
    hq0m = hq0c;
    hq1m = hq1c;
    hq0c = hq0n;
    hq1c = hq1n;
    if (DECIDE && ((rows >> h) & 1u)) {  // wave-uniform: rows holding an anyon
      add_moves(mv, 0, h, decide_site(b.P0[h], b.Q0[h], (b.s0 >> h) & 1u));
      add_moves(mv, 1, h, decide_site(b.P1[h], b.Q1[h], (b.s1 >> h) & 1u));
    }
  }
}

// Feedback for the band: link flips from the moves (OR of both endpoints,
// eq. (ddfeedback)) and the syndrome update.  MB is an LDS array [wave][64]
// used to pass the y-moves across wave boundaries.  xo[c] receives the
// flipped x-links to the right of column c, yo[c] the flipped y-links above
// each row of column c.
template <int H>
__device__ __forceinline__ void band_feedback(BandLane<H> &b, const Moves &mv, uint4 *MB, int w, int wdn,
                                              int wup, int lane, uint32_t (&xo)[2], uint32_t (&yo)[2]) {
  MB[w * 64 + lane] = make_uint4(mv.py[0], mv.py[1], mv.my[0], mv.my[1]);
  __syncthreads();
  const uint4 upm = MB[wup * 64 + lane];  // wave above: bit 0 of its my = its first row moves -y
  const uint4 dnm = MB[wdn * 64 + lane];  // wave below: bit H-1 of its py = its last row moves +y
  constexpr uint32_t F = full_mask<H>();
  // x-links: column 2i -> 2i+1 and column 2i+1 -> 2i+2 (next lane's column 2i)
  xo[0] = mv.px[0] | mv.mx[1];
  xo[1] = mv.px[1] | from_right(mv.mx[0]);
  const uint32_t xl0 = from_left(xo[1]), xl1 = xo[0];
  {
    const uint32_t yd = ((mv.py[0] << 1) | ((dnm.x >> (H - 1)) & 1u) | mv.my[0]) & F;
    yo[0] = (mv.py[0] | (mv.my[0] >> 1) | ((upm.z & 1u) << (H - 1))) & F;
    b.s0 = (b.s0 ^ xo[0] ^ xl0 ^ yo[0] ^ yd) & F;
  }
  {
    const uint32_t yd = ((mv.py[1] << 1) | ((dnm.y >> (H - 1)) & 1u) | mv.my[1]) & F;
    yo[1] = (mv.py[1] | (mv.my[1] >> 1) | ((upm.w & 1u) << (H - 1))) & F;
    b.s1 = (b.s1 ^ xo[1] ^ xl1 ^ yo[1] ^ yd) & F;
  }
}

}  // namespace mpd
