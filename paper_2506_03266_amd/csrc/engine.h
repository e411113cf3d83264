// engine.h -- device-side building blocks of the decoder sweep (gfx950).
//
// One thread owns a vertical strip of H consecutive rows in one column of a
// rectangular region of the lattice (the whole lattice for small L, a tile
// plus halo for large L).  It keeps its sites' four message registers in
// VGPRs and its syndrome bits in one 32-bit mask; neighbours are exchanged
// through LDS.
//
// Message registers are stored as emission times instead of the paper's
// distances: for a register holding m > 0 after sub-step s the stored value
// is e = s - m + 1 (e = 0 for "no message").  The rule A^{(D)} of
// Def. "message passing automaton, general dimensions" (Sec. 3.2) -- 1 if an
// anyon sits on the line C^{(a)}_{r - s a}, else the minimum of the nonzero
// registers on that line plus one, else 0 -- then reads
//     e'(r) = max over q on the line of ( sigma_q ? s : e(q) ),
// because a smaller nonzero m is a larger e, "no message" (0) is the
// smallest e, and an anyon emits at the current sub-step s, which exceeds
// every stored time.  So one sub-step is a 3-wide max of packed u16 pairs.
// Values stay exact while s <= 65535.
//
// Packed layout of a site: P = e^{+x} | e^{-x} << 16, Q = e^{+y} | e^{-y} << 16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpd {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pmax(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(
      uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}

__device__ __forceinline__ uint32_t pmax3(uint32_t a, uint32_t b, uint32_t c) {
  return pmax(pmax(a, b), c);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with counter (c0, c1, c2, 0).
struct Words4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t k0, uint32_t k1, uint32_t c1 = 0u,
                                                uint32_t c2 = 0u) {
  uint32_t c3 = 0u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product each (v_mad_u64_u32) instead of separate lo/hi multiplies
    const uint64_t m0 = (uint64_t)0xD2511F53u * c0, m1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)m0, hi0 = (uint32_t)(m0 >> 32);
    const uint32_t lo1 = (uint32_t)m1, hi1 = (uint32_t)(m1 >> 32);
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);  // 3-way XOR
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// floor(p 2^32) clamped to [0, 2^32]; exact in double, so identical to the
// host's value for the same p.
__device__ __forceinline__ uint64_t device_threshold(double p) {
  double t = floor(p * 4294967296.0);
  t = t < 0.0 ? 0.0 : (t > 4294967296.0 ? 4294967296.0 : t);
  return (uint64_t)t;
}

// Link flips of site i = y*L + x from its Philox words (x-link, y-link).
__device__ __forceinline__ void site_noise(uint32_t i, uint32_t k0, uint32_t k1, uint64_t thr,
                                           bool &fx, bool &fy) {
  const Words4 w = philox4x32_10(i >> 1, k0, k1);
  const uint32_t wx = (i & 1u) ? w.w2 : w.w0;
  const uint32_t wy = (i & 1u) ? w.w3 : w.w1;
  fx = (uint64_t)wx < thr;
  fy = (uint64_t)wy < thr;
}

// Limited-memory variant of the rule (Sec. 5.3, corollary on limited
// classical memory).  With a finite m_max a message whose value would exceed
// m_max disappears.  In emission-time form a register is live after sub-step
// s iff e >= s + 1 - m_max: a dropped message keeps a stale emission time
// that is smaller than every live one, so the 3-wide maxima of the update
// stay exact and only the decision has to ignore registers below the
// threshold.  With u > 0, every u-th decoder step t (from 1) moves each
// anyon in a random direction instead: Philox4x32-10 keyed by the sample's
// seed, counter (i >> 1, t, MOVE_TAG, 0), word (i & 1) of site i, mod 4 ->
// +x, -x, +y, -y.
constexpr uint32_t MOVE_TAG = 0x4D4F5645u;

// Smallest live emission time after sub-step s (1 with no truncation).
__device__ __forceinline__ uint32_t live_threshold(uint32_t s, int m_max) {
  return (m_max > 0 && s + 1u > (uint32_t)m_max + 1u) ? s + 1u - (uint32_t)m_max : 1u;
}

// Random directions of the two sites of a generator pair (word 0: the even
// site 2q, word 1: the odd site 2q + 1): 0 +x, 1 -x, 2 +y, 3 -y.
__device__ __forceinline__ uint2 random_dirs(uint32_t pair, uint32_t t, uint32_t k0, uint32_t k1) {
  const Words4 w = philox4x32_10(pair, k0, k1, t, MOVE_TAG);
  return make_uint2(w.w0 & 3u, w.w1 & 3u);
}

// Per-thread view of the region.
struct Geo {
  int RX;          // region width (columns)
  int c, j, y0;    // own column, strip index, first row of the strip
  int cl, cr;      // left / right neighbour columns (wrapped or clamped)
  int jd, ju;      // strip below / above (wrapped or clamped)
  int rowDn, rowUp;  // region rows just below / above the strip
};

// Rows between scheduling fences in the sub-step loop.
constexpr int SCHED_ROWS = 4;

template <int H>
__device__ __forceinline__ constexpr uint32_t full_mask() {
  return H >= 32 ? 0xFFFFFFFFu : ((1u << H) - 1u);
}

// One application of A^{(D)} to all four registers of every site (all
// threads of the block together).  sub-step time s is passed packed as
// ss = s | s << 16.  F is the LDS exchange buffer (one uint2 per site).
// With OPEN, a thread of a rough-boundary column (inB) publishes "emits now"
// in P, so that its neighbours' x-registers read a message of value 1, and
// nothing in Q.
template <int H, bool OPEN = false>
__device__ __forceinline__ void substep(uint32_t (&P)[H], uint32_t (&Q)[H], uint32_t sig, uint32_t ss,
                                        uint2 *F, const Geo &g, bool inB = false) {
  const int RX = g.RX;
  // Opaque copies of the column indices: every row address below is then
  // formed where it is used instead of being hoisted out of the decoder loop
  // (with a run-time row stride each row would hold its own address VGPRs).
  int gc = g.c, gcl = g.cl, gcr = g.cr;
  asm volatile("" : "+v"(gc), "+v"(gcl), "+v"(gcr));
  // publish the folded values: an anyon site reads as "emits now"
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const bool a = (sig >> h) & 1u;
    F[(g.y0 + h) * RX + gc] =
        (OPEN && inB) ? make_uint2(ss, 0u) : make_uint2(a ? ss : P[h], a ? ss : Q[h]);
  }
  __syncthreads();
  // Rolling window over region rows y0-1 .. y0+H.  For row r:
  //   pl/pr = P of the left/right column (vertical max feeds +x / -x),
  //   hq    = max of Q over columns x-1, x, x+1 (feeds +y from row below,
  //           -y from row above).
  uint32_t pl2, pl1, pr2, pr1, hq2, hq1;
  {
    const uint2 a = F[g.rowDn * RX + gcl], b = F[g.rowDn * RX + gcr];
    const uint32_t q = F[g.rowDn * RX + gc].y;
    pl2 = a.x;
    pr2 = b.x;
    hq2 = pmax3(a.y, q, b.y);
  }
  {
    const uint2 a = F[g.y0 * RX + gcl], b = F[g.y0 * RX + gcr];
    const uint32_t q = (sig & 1u) ? ss : Q[0];
    pl1 = a.x;
    pr1 = b.x;
    hq1 = pmax3(a.y, q, b.y);
  }
#pragma unroll
  for (int i = 2; i <= H + 1; ++i) {
    uint2 a, b;
    uint32_t q;
    if (i <= H) {
      const int r = g.y0 + i - 1;
      a = F[r * RX + gcl];
      b = F[r * RX + gcr];
      q = ((sig >> (i - 1)) & 1u) ? ss : Q[i - 1];
    } else {
      a = F[g.rowUp * RX + gcl];
      b = F[g.rowUp * RX + gcr];
      q = F[g.rowUp * RX + gc].y;
    }
    const uint32_t pl0 = a.x, pr0 = b.x, hq0 = pmax3(a.y, q, b.y);
    const int h = i - 2;
    const uint32_t vl = pmax3(pl2, pl1, pl0), vr = pmax3(pr2, pr1, pr0);
    P[h] = (vl & 0xFFFFu) | (vr & 0xFFFF0000u);
    Q[h] = (hq2 & 0xFFFFu) | (hq0 & 0xFFFF0000u);
    pl2 = pl1;
    pl1 = pl0;
    pr2 = pr1;
    pr1 = pr0;
    hq2 = hq1;
    hq1 = hq0;
    // keep at most a few rows of LDS loads in flight (bounded VGPR use)
    if ((i & (SCHED_ROWS - 1)) == SCHED_ROWS - 1) __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
}

// Feedback F^{(D)} for the strip.  Each anyon picks the register with the
// smallest nonzero distance (largest emission time), ties broken in the
// order -y < -x < +x < +y (argmin' of eq. (degbreak)); it moves one link
// toward that message's source unless the opposite register on the same
// axis is equal (force sgn(0) = 0).  A link flips if either endpoint moves
// across it (OR of eq. (ddfeedback)).  Returns the new syndrome mask; xo
// and yo receive the flipped x-links (x,y)-(x+1,y) and y-links
// (x,y)-(x,y+1) of the strip, for the correction winding.
// `ethr` is the smallest live emission time (live_threshold); with `rnd`
// (a random-move step t of the limited-memory variant) every anyon of the
// strip moves in its random direction instead, drawn with key (k0, k1) for
// site i = row * L + g.c.
template <int H, bool RULE>
__device__ __forceinline__ uint32_t feedback(const uint32_t (&P)[H], const uint32_t (&Q)[H], uint32_t sig,
                                             uint4 *MV, const Geo &g, uint32_t &xo, uint32_t &yo, uint32_t ethr,
                                             bool rnd, uint32_t t, uint32_t k0, uint32_t k1, int L) {
  uint32_t mpx = 0u, mmx = 0u, mpy = 0u, mmy = 0u;
  if (RULE && sig && rnd) {
    for (int h = 0; h < H; ++h) {
      if ((sig >> h) & 1u) {
        const uint32_t i = (uint32_t)((g.y0 + h) * L + g.c);
        const uint2 d = random_dirs(i >> 1, t, k0, k1);
        const uint32_t dir = (i & 1u) ? d.y : d.x;
        const uint32_t bit = 1u << h;
        mpx |= dir == 0u ? bit : 0u;
        mmx |= dir == 1u ? bit : 0u;
        mpy |= dir == 2u ? bit : 0u;
        mmy |= dir == 3u ? bit : 0u;
      }
    }
  } else if (sig) {
#pragma unroll
    for (int h = 0; h < H; ++h) {
      if ((sig >> h) & 1u) {
        const uint32_t px = P[h] & 0xFFFFu, mx = P[h] >> 16;
        const uint32_t py = Q[h] & 0xFFFFu, my = Q[h] >> 16;
        const uint32_t M = max(max(px, mx), max(py, my));
        const uint32_t bit = 1u << h;
        if (M >= ethr) {  // some live message (M != 0 without truncation)
          if (my == M) {
            if (py != M) mpy |= bit;   // -y message: source above, move +y
          } else if (mx == M) {
            if (px != M) mpx |= bit;   // -x message: source right, move +x
          } else if (px == M) {
            mmx |= bit;                // +x message: source left, move -x
          } else {
            mmy |= bit;                // +y message: source below, move -y
          }
        }
      }
    }
  }
  MV[g.j * g.RX + g.c] = make_uint4(mpx, mmx, mpy, mmy);
  __syncthreads();
  const uint4 R = MV[g.j * g.RX + g.cr], Lf = MV[g.j * g.RX + g.cl];
  const uint4 U = MV[g.ju * g.RX + g.c], D = MV[g.jd * g.RX + g.c];
  constexpr uint32_t FULL = full_mask<H>();
  xo = mpx | R.y;                                                      // link to the right
  const uint32_t xl = Lf.x | mmx;                                      // link to the left
  yo = (mpy | (mmy >> 1) | ((U.w & 1u) << (H - 1))) & FULL;           // link upward
  const uint32_t yd = ((mpy << 1) | ((D.z >> (H - 1)) & 1u) | mmy) & FULL;  // link downward
  return (sig ^ xo ^ xl ^ yo ^ yd) & FULL;
}

// Syndrome of the strip from its link bits: sigma = ex ^ ex(left) ^ ey ^ ey(below).
template <int H>
__device__ __forceinline__ uint32_t syndrome_from_links(uint32_t exb, uint32_t eyb, uint4 *MV,
                                                        const Geo &g) {
  MV[g.j * g.RX + g.c] = make_uint4(exb, eyb, 0u, 0u);
  __syncthreads();
  const uint32_t exl = MV[g.j * g.RX + g.cl].x;
  const uint32_t eyd = MV[g.jd * g.RX + g.c].y;
  __syncthreads();
  constexpr uint32_t FULL = full_mask<H>();
  return (exb ^ exl ^ eyb ^ ((eyb << 1) | ((eyd >> (H - 1)) & 1u))) & FULL;
}

}  // namespace mpd
