// mpd.hip -- kernels and C ABI of the MI355X decoder (see include/mpd.h).
//
// Two execution shapes share the device engine of engine.h:
//  * resident: one workgroup holds a whole L x L sample in LDS/VGPRs and runs
//    it from noise to termination with no HBM traffic for the state
//    (L <= 128 with a strip height dividing L; at L = 64 and 128 the
//    bit-sliced kernel of bits.h runs the first ten steps before it);
//  * band (L >= 256, multiples of 16): each workgroup holds a region of 128
//    columns x 256 rows in VGPRs (band.h), of which all but a halo of 4k
//    columns (and 4k rows rounded up to 16, unless the region spans the
//    lattice height) on each side are its own (k = decoder steps per pass:
//    a step moves information by v = 3 sites for the messages plus 1 for
//    the feedback); it runs k steps on chip and writes its own sites back to
//    HBM.  A separate kernel draws the noise and the initial syndrome once.
//    Between passes a small kernel turns the per-step "anyons left" bits
//    into T_dec and compacts the list of unfinished samples; each sample
//    keeps its own step count, so groups of samples may start with passes
//    of different depth (learned scheduling, cnn.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "band.h"
#include "engine.h"
#include "host.h"
#include "mpd.h"
#include "torus.h"

namespace mpd {

// ---------------------------------------------------------------------------
// Resident kernel: one workgroup per sample.
// ---------------------------------------------------------------------------

struct ResidentArgs {
  int L;
  int64_t n;
  const uint64_t *seeds;   // seeded mode when links == nullptr
  uint64_t thr;            // flip threshold floor(p 2^32) when p_arr == nullptr
  const double *p_arr;     // per-sample noise strength (mixed batches) or nullptr
  const uint32_t *links;   // explicit error patterns
  int T_max;
  int t_exact;             // >= 0: run exactly this many steps (state export)
  int32_t *T_dec;
  uint8_t *flags;
  uint32_t *syn;           // final syndrome bits (may be null)
  int16_t *m_out;          // state export (t_exact >= 0)
  uint8_t *wind_out;
  int m_max;               // limited-memory variant: 0 = no truncation
  int u;                   // random moves every u steps, 0 = none
  const uint64_t *move_seeds;  // keys of the random moves in explicit-error mode
  int open;                // 1: open lattice (rough left / right columns)
  // resume from an exported state (torus): registers [n][4][L*L] in distance
  // form, syndrome bits and winding bits after t_start steps
  const int16_t *m_in;
  const uint32_t *syn_in;
  const uint8_t *wind_in;
  int t_start;
};

// Kernel variants of the resident decoder: the plain rule, the
// limited-memory rule (m_max, u), and the open lattice.
enum ResidentMode { RES_PLAIN = 0, RES_RULE = 1, RES_OPEN = 2 };

__device__ __forceinline__ uint32_t parity32(uint32_t x) { return __popc(x) & 1u; }

// MODE RES_RULE compiles in the limited-memory variant (a.m_max, a.u).
// MODE RES_OPEN decodes on the open lattice of the appendix on open
// boundaries: sites (x, y) without wrap; the columns x = 0 and x = L-1 are
// the rough boundary B (no syndrome, no messages; they source x-messages
// into the bulk and absorb anyons); rows y = 0 and y = L-1 end smooth.
// Qubits are the links with a bulk endpoint (x-links for x <= L-2, y-links
// for y <= L-2 in bulk columns); bits of other links are ignored.  The
// region keeps one extra LDS row of zeros that the bottom and top strips
// read as their outer neighbour row, which clips every line at the smooth
// edges; B columns publish "emits now" in P (so their x-messages enter the
// bulk) and 0 in Q.  One logical qubit: the correction and error windings
// are read on the x-links from column L-2 to L-1.
template <int H, int MODE>
__global__ __launch_bounds__(1024) void k_resident(ResidentArgs a) {
  constexpr bool RULE = MODE == RES_RULE, OPEN = MODE == RES_OPEN;
  extern __shared__ __align__(16) unsigned char smem[];
  const int L = a.L, RX = L, NS = L / H;
  uint2 *F = reinterpret_cast<uint2 *>(smem);
  uint4 *MV = reinterpret_cast<uint4 *>(smem + (size_t)RX * (OPEN ? L + 1 : L) * sizeof(uint2));
  uint32_t *red = reinterpret_cast<uint32_t *>(MV + (size_t)RX * NS);
  const int64_t sample = blockIdx.x;
  const int tid = threadIdx.x;

  Geo g;
  g.RX = RX;
  g.c = tid % RX;
  g.j = tid / RX;
  g.y0 = g.j * H;
  g.cl = g.c == 0 ? RX - 1 : g.c - 1;
  g.cr = g.c == RX - 1 ? 0 : g.c + 1;
  g.jd = g.j == 0 ? NS - 1 : g.j - 1;
  g.ju = g.j == NS - 1 ? 0 : g.j + 1;
  g.rowDn = g.y0 == 0 ? (OPEN ? L : L - 1) : g.y0 - 1;
  g.rowUp = g.y0 + H == L ? (OPEN ? L : 0) : g.y0 + H;
  const bool inB = OPEN && (g.c == 0 || g.c == L - 1);  // rough boundary column
  if (OPEN && g.j == 0) F[(size_t)L * RX + g.c] = make_uint2(0u, 0u);  // the zero row

  if (tid == 0) red[0] = 0u;

  uint32_t P[H], Q[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    P[h] = 0u;
    Q[h] = 0u;
  }
  uint32_t wind = 0u;  // bit0 Wx(E), bit1 Wy(E), bit2 Wx(C), bit3 Wy(C)
  uint32_t sig = 0u;
  const uint32_t t0 = a.syn_in != nullptr ? (uint32_t)a.t_start : 0u;  // steps already run
  if (a.syn_in != nullptr) {
    // ---- resume: syndrome bits, registers (distance m -> emission time
    // 3 t0 - m + 1) and the winding bits of the exported state
    const int64_t n2 = (int64_t)L * L, nw = (n2 + 31) / 32;
    const int16_t *mi = a.m_in + sample * 4 * n2;
    const uint32_t s0 = 3u * t0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int64_t i = (int64_t)(g.y0 + h) * L + g.c;
      sig |= ((a.syn_in[sample * nw + (i >> 5)] >> (i & 31)) & 1u) << h;
      uint32_t e[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const uint32_t m = (uint32_t)(uint16_t)mi[d * n2 + i];
        e[d] = m != 0u ? ((s0 - m + 1u) & 0xFFFFu) : 0u;
      }
      P[h] = e[0] | e[1] << 16;
      Q[h] = e[2] | e[3] << 16;
    }
    if (tid == 0) wind = a.wind_in[sample] & 15u;
  } else {
  // ---- noise / error pattern -> link bits of the strip
  uint32_t exb = 0u, eyb = 0u;
  if (a.links == nullptr) {
    const uint64_t seed = a.seeds[sample];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint64_t thr = a.p_arr ? device_threshold(a.p_arr[sample]) : a.thr;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      bool fx, fy;
      site_noise((uint32_t)((g.y0 + h) * L + g.c), k0, k1, thr, fx, fy);
      exb |= (uint32_t)fx << h;
      eyb |= (uint32_t)fy << h;
      if (h & 1) __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    const int64_t lw = (2 * (int64_t)L * L + 31) / 32;
    const uint32_t *w = a.links + sample * lw;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const uint32_t lx = 2u * (uint32_t)((g.y0 + h) * L + g.c), ly = lx + 1u;
      exb |= ((w[lx >> 5] >> (lx & 31u)) & 1u) << h;
      eyb |= ((w[ly >> 5] >> (ly & 31u)) & 1u) << h;
    }
  }
  if (OPEN) {  // drop the links that do not exist on the open lattice
    if (g.c == L - 1) exb = 0u;
    if (inB) eyb = 0u;
    if (g.j == NS - 1) eyb &= ~(1u << (H - 1));
  }
  if (g.c == (OPEN ? L - 2 : L - 1)) wind ^= parity32(exb);
  if (!OPEN && g.j == NS - 1) wind ^= ((eyb >> (H - 1)) & 1u) << 1;
  sig = syndrome_from_links<H>(exb, eyb, MV, g);
  if (inB) sig = 0u;
  }

  int alive = __syncthreads_or(sig != 0u);
  const bool exact = a.t_exact >= 0;
  const int steps = exact ? a.t_exact : a.T_max;
  uint32_t mk0 = 0u, mk1 = 0u;  // key of the random moves
  if (RULE && a.u > 0) {
    // seeded decodes move with their noise seed; explicit errors and resumed
    // states with their move seeds
    const uint64_t ms = (a.links == nullptr && a.syn_in == nullptr) ? a.seeds[sample] : a.move_seeds[sample];
    mk0 = (uint32_t)ms;
    mk1 = (uint32_t)(ms >> 32);
  }
  int t = 0;
  while (t < steps && (exact || alive)) {
#pragma unroll 1
    for (int sub = 1; sub <= 3; ++sub) {
      const uint32_t s = 3u * (t0 + (uint32_t)t) + (uint32_t)sub;
      substep<H, OPEN>(P, Q, sig, s | (s << 16), F, g, inB);
    }
    uint32_t xo, yo;
    const uint32_t t1 = t0 + (uint32_t)(t + 1);
    if (RULE) {
      const bool rnd = a.u > 0 && t1 % (uint32_t)a.u == 0u;
      sig = feedback<H, true>(P, Q, sig, MV, g, xo, yo, live_threshold(3u * t1, a.m_max), rnd, t1, mk0, mk1, L);
    } else {
      sig = feedback<H, false>(P, Q, sig, MV, g, xo, yo, 1u, false, t1, 0u, 0u, L);
    }
    if (inB) sig = 0u;  // an anyon moved onto B is absorbed
    if (g.c == (OPEN ? L - 2 : L - 1)) wind ^= parity32(xo) << 2;
    if (!OPEN && g.j == NS - 1) wind ^= ((yo >> (H - 1)) & 1u) << 3;
    ++t;
    alive = __syncthreads_or(sig != 0u);
  }

  // ---- reduce the winding bits of the block
  if (wind) atomicXor(&red[0], wind);
  __syncthreads();
  const uint32_t W = red[0];

  const int64_t nw = ((int64_t)L * L + 31) / 32;
  uint32_t *out_bits = exact ? a.syn : a.syn;
  if (out_bits != nullptr) {
    uint32_t *SW = reinterpret_cast<uint32_t *>(F);  // F is free now
    for (int w = tid; w < nw; w += blockDim.x) SW[w] = 0u;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < H; ++h)
      if ((sig >> h) & 1u) {
        const uint32_t i = (uint32_t)((g.y0 + h) * L + g.c);
        atomicOr(&SW[i >> 5], 1u << (i & 31u));
      }
    __syncthreads();
    for (int w = tid; w < nw; w += blockDim.x) out_bits[sample * nw + w] = SW[w];
  }

  if (exact) {
    if (a.m_out != nullptr) {
      const uint32_t snow = 3u * (t0 + (uint32_t)a.t_exact);
      const uint32_t live = RULE ? live_threshold(snow, a.m_max) : 1u;
      const int64_t n2 = (int64_t)L * L;
      int16_t *mo = a.m_out + sample * 4 * n2;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int64_t i = (int64_t)(g.y0 + h) * L + g.c;
        const uint32_t e[4] = {P[h] & 0xFFFFu, P[h] >> 16, Q[h] & 0xFFFFu, Q[h] >> 16};
#pragma unroll
        for (int d = 0; d < 4; ++d) mo[d * n2 + i] = (int16_t)(e[d] >= live && !inB ? (snow - e[d] + 1u) : 0u);
      }
    }
    if (tid == 0 && a.wind_out != nullptr) a.wind_out[sample] = (uint8_t)W;
  } else if (tid == 0) {
    const uint32_t fail = ((W ^ (W >> 2)) & 3u) != 0u;
    const uint32_t timeout = alive ? 1u : 0u;
    a.T_dec[sample] = t;
    a.flags[sample] = (uint8_t)((fail | timeout) | (timeout << 1));
  }
}

// ---------------------------------------------------------------------------
// Whole-lattice band kernel for L = 64 and L = 128 (seeded, plain rule).
// ---------------------------------------------------------------------------

struct TorusArgs {
  int64_t n;
  const uint64_t *seeds;
  uint64_t thr;          // flip threshold when p_arr == nullptr
  const double *p_arr;   // per-sample noise strength (mixed batches) or nullptr
  int T_max;
  int32_t *T_dec;
  uint8_t *flags;
  uint32_t *syn;         // final syndrome bits (may be null)
  int resume = 0;        // nonzero: only samples with T_dec[sample] < 0 (left by k_bits)
};

// One workgroup per sample, the whole L x L torus in registers: NW waves of
// 16-row strips; a lane holds CPL adjacent columns (CPL = 1: L = 64, CPL = 2:
// L = 128, 64 lanes span the width).  The periodic wrap in x is a wave-wide
// DPP rotation and the wrap in y the wave order, so nothing is halo and the
// state never leaves the chip; per decoder step only the strips' edge rows
// and edge moves go through LDS.  Noise, syndrome, decoder steps until no
// anyon is left (one block-wide OR per step), classification and the final
// syndrome, in one launch (Def. "synchronous automaton decoder"; the rule of
// Def. "message passing automaton, general dimensions" as in engine.h).
template <int CPL, int NW>
__global__ __launch_bounds__(NW * 64) void k_torus(TorusArgs a) {
  constexpr int H = 16, L = 64 * CPL;
  constexpr uint32_t F = full_mask<H>();
  extern __shared__ __align__(16) unsigned char smem[];
  using Slot = typename std::conditional<CPL == 2, uint4, uint2>::type;
  Slot *BND0 = reinterpret_cast<Slot *>(smem);  // two sub-step slots [NW][2][64]
  Slot *BND1 = BND0 + NW * 2 * 64;
  uint2 *MB = reinterpret_cast<uint2 *>(BND1 + NW * 2 * 64);  // [NW][64]
  __shared__ uint32_t red;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wdn = w == 0 ? NW - 1 : w - 1, wup = w == NW - 1 ? 0 : w + 1;
  // one sample per workgroup, or (resume) a grid of resident workgroups
  // stepping over the samples that the bit-sliced kernel left
  for (int64_t sample = blockIdx.x; sample < a.n; sample += gridDim.x) {
    if (a.resume && a.T_dec[sample] >= 0) continue;  // decoded by the bit-sliced kernel
    __syncthreads();  // the previous sample's last reads of LDS are done
    const uint64_t seed = a.seeds[sample];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint64_t thr = a.p_arr ? device_threshold(a.p_arr[sample]) : a.thr;
    const int y0 = w * H;
    if (threadIdx.x == 0) red = 0u;
    uint32_t wind = 0u;  // bit0 Wx(E), bit1 Wy(E), bit2 Wx(C), bit3 Wy(C)
    int t = 0, alive;
    uint32_t s0 = 0u, s1 = 0u;  // syndrome masks (s1: second column, CPL = 2)

    if constexpr (CPL == 2) {
      BandLane<H> b;
#pragma unroll
      for (int h = 0; h < H; ++h) b.P0[h] = b.Q0[h] = b.P1[h] = b.Q1[h] = 0u;
      // noise: columns 2 lane, 2 lane + 1 of rows y0 .. y0 + 15 (one generator block per site pair)
      uint32_t ex0 = 0u, ey0 = 0u, ex1 = 0u, ey1 = 0u;
#pragma unroll 4
      for (int h = 0; h < H; ++h) {
        const Words4 r = philox4x32_10((uint32_t)((y0 + h) * (L / 2) + lane), k0, k1);
        ex0 |= (uint32_t)((uint64_t)r.w0 < thr) << h;
        ey0 |= (uint32_t)((uint64_t)r.w1 < thr) << h;
        ex1 |= (uint32_t)((uint64_t)r.w2 < thr) << h;
        ey1 |= (uint32_t)((uint64_t)r.w3 < thr) << h;
      }
      MB[w * 64 + lane] = make_uint2((ey0 >> (H - 1)) & 1u, (ey1 >> (H - 1)) & 1u);  // top-row y-links
      __syncthreads();
      const uint2 eyd = MB[wdn * 64 + lane];  // y-links of the row below the strip
      const uint32_t exl = from_left<true>(ex1);
      b.s0 = (ex0 ^ exl ^ ey0 ^ ((ey0 << 1) | eyd.x)) & F;
      b.s1 = (ex1 ^ ex0 ^ ey1 ^ ((ey1 << 1) | eyd.y)) & F;
      if (lane == 63) wind ^= __popc(ex1) & 1u;                           // x-links leaving column L-1
      if (w == NW - 1) wind ^= (((ey0 ^ ey1) >> (H - 1)) & 1u) << 1;      // y-links leaving row L-1
      alive = __syncthreads_or((b.s0 | b.s1) != 0u);
      while (t < a.T_max && alive) {
        const uint32_t t3 = 3u * (uint32_t)t;
        const uint32_t rows = wave_rows<H>(b.s0, b.s1);
        Moves mv = {0u, 0u, 0u, 0u};
        uint4 *sa = (t & 1) ? BND1 : BND0, *sb = (t & 1) ? BND0 : BND1;
        if (rows) band_fold<H>(b, (t3 + 1u) | ((t3 + 1u) << 16), rows);
        band_substep<H, false, true>(b, sa, w, wdn, wup, lane, rows, 1u, mv);
        if (rows) band_fold<H>(b, (t3 + 2u) | ((t3 + 2u) << 16), rows);
        band_substep<H, false, true>(b, sb, w, wdn, wup, lane, rows, 1u, mv);
        if (rows) band_fold<H>(b, (t3 + 3u) | ((t3 + 3u) << 16), rows);
        band_substep<H, true, true>(b, sa, w, wdn, wup, lane, rows, 1u, mv);
        uint32_t xo[2], yo[2];
        band_feedback<H, true>(b, mv, MB, w, wdn, wup, lane, xo, yo);
        if (lane == 63) wind ^= (__popc(xo[1]) & 1u) << 2;
        if (w == NW - 1) wind ^= (((yo[0] ^ yo[1]) >> (H - 1)) & 1u) << 3;
        ++t;
        alive = __syncthreads_or((b.s0 | b.s1) != 0u);
      }
      s0 = b.s0;
      s1 = b.s1;
    } else {
      uint32_t P[H], Q[H];
#pragma unroll
      for (int h = 0; h < H; ++h) P[h] = Q[h] = 0u;
      // noise: column x = lane of rows y0 .. y0 + 15.  The two lanes of a site
      // pair share generator blocks: for each row pair (h, h + 1) the even lane
      // draws row h's block and the odd lane row h + 1's, and they swap the
      // words of the other site (DPP quad_perm [1, 0, 3, 2]).
      uint32_t ex = 0u, ey = 0u;
      const uint32_t q = (uint32_t)lane & 1u;
#pragma unroll 2
      for (int h = 0; h < H; h += 2) {
        const Words4 r = philox4x32_10((uint32_t)((y0 + h + (int)q) * (L / 2) + (lane >> 1)), k0, k1);
        const uint32_t ownx = q ? r.w2 : r.w0, owny = q ? r.w3 : r.w1;  // this lane's site in row h + q
        const uint32_t sendx = q ? r.w0 : r.w2, sendy = q ? r.w1 : r.w3;  // the partner's site in that row
        const uint32_t gotx = (uint32_t)__builtin_amdgcn_mov_dpp((int)sendx, 0xB1, 0xF, 0xF, false);
        const uint32_t goty = (uint32_t)__builtin_amdgcn_mov_dpp((int)sendy, 0xB1, 0xF, 0xF, false);
        const uint32_t x0 = q ? gotx : ownx, y0w = q ? goty : owny;  // row h
        const uint32_t x1 = q ? ownx : gotx, y1w = q ? owny : goty;  // row h + 1
        ex |= ((uint32_t)((uint64_t)x0 < thr) << h) | ((uint32_t)((uint64_t)x1 < thr) << (h + 1));
        ey |= ((uint32_t)((uint64_t)y0w < thr) << h) | ((uint32_t)((uint64_t)y1w < thr) << (h + 1));
      }
      MB[w * 64 + lane] = make_uint2((ey >> (H - 1)) & 1u, 0u);
      __syncthreads();
      const uint32_t eyd = MB[wdn * 64 + lane].x;
      s0 = (ex ^ from_left<true>(ex) ^ ey ^ ((ey << 1) | eyd)) & F;
      if (lane == 63) wind ^= __popc(ex) & 1u;
      if (w == NW - 1) wind ^= ((ey >> (H - 1)) & 1u) << 1;
      alive = __syncthreads_or(s0 != 0u);
      while (t < a.T_max && alive) {
        const uint32_t t3 = 3u * (uint32_t)t;
        const uint32_t rows = wave_rows<H>(s0, 0u);
        Moves mv = {0u, 0u, 0u, 0u};
        uint2 *sa = (t & 1) ? BND1 : BND0, *sb = (t & 1) ? BND0 : BND1;
        if (rows) col_fold<H>(P, Q, s0, (t3 + 1u) | ((t3 + 1u) << 16), rows);
        col_substep<H, false>(P, Q, s0, sa, w, wdn, wup, lane, rows, 1u, mv);
        if (rows) col_fold<H>(P, Q, s0, (t3 + 2u) | ((t3 + 2u) << 16), rows);
        col_substep<H, false>(P, Q, s0, sb, w, wdn, wup, lane, rows, 1u, mv);
        if (rows) col_fold<H>(P, Q, s0, (t3 + 3u) | ((t3 + 3u) << 16), rows);
        col_substep<H, true>(P, Q, s0, sa, w, wdn, wup, lane, rows, 1u, mv);
        uint32_t xo, yo;
        s0 = col_feedback<H>(s0, mv, MB, w, wdn, wup, lane, xo, yo);
        if (lane == 63) wind ^= (__popc(xo) & 1u) << 2;
        if (w == NW - 1) wind ^= ((yo >> (H - 1)) & 1u) << 3;
        ++t;
        alive = __syncthreads_or(s0 != 0u);
      }
    }

    // winding bits of the block, classification, final syndrome
    if (wind) atomicXor(&red, wind);
    __syncthreads();
    const uint32_t W = red;
    if (a.syn != nullptr) {
      constexpr int NWORD = L * L / 32;
      uint32_t *SW = reinterpret_cast<uint32_t *>(smem);  // the sub-step slots are free now
      for (int i = threadIdx.x; i < NWORD; i += blockDim.x) SW[i] = 0u;
      __syncthreads();
      if (s0 | s1)
        for (int h = 0; h < H; ++h)
          for (int c = 0; c < CPL; ++c)
            if ((((c ? s1 : s0) >> h) & 1u)) {
              const uint32_t i = (uint32_t)((y0 + h) * L + CPL * lane + c);
              atomicOr(&SW[i >> 5], 1u << (i & 31u));
            }
      __syncthreads();
      for (int i = threadIdx.x; i < NWORD; i += blockDim.x) a.syn[sample * NWORD + i] = SW[i];
    }
    if (threadIdx.x == 0) {
      const uint32_t fail = ((W ^ (W >> 2)) & 3u) != 0u;
      const uint32_t timeout = alive ? 1u : 0u;
      a.T_dec[sample] = t;
      a.flags[sample] = (uint8_t)((fail | timeout) | (timeout << 1));
    }
  }
}

// ---------------------------------------------------------------------------
// Band path: regions of 128 columns x 256 rows, k steps per pass.
// ---------------------------------------------------------------------------

constexpr int BAND_H = 16;                 // rows per wave
constexpr int BAND_NW = 16;                // waves per workgroup (full-size regions)
constexpr int BAND_NW_SMALL = 4;           // waves per workgroup for passes that underfill the GPU
constexpr int BAND_RX = 128;               // region columns (2 per lane)
constexpr int BAND_RY = BAND_NW * BAND_H;  // region rows (full-size regions)
constexpr int TILE_H = BAND_H;             // rows per syndrome word pair in HBM
constexpr int BAND_MAX_N = 65535;          // samples per band-path pass (grid y dimension)

}  // namespace mpd

#include "bits.h"

namespace mpd {

struct BandArgs {
  int L;
  int write_state;  // 0: do not store the state (samples expected to finish in this pass)
  int k;            // decoder steps in this pass (fewer for a sample that reaches T_max)
  int T_max;
  const int32_t *t_done;  // per sample: steps already done (0: registers start empty)
  int hx, tx;       // column halo, owned columns per tile
  int hy, ty;       // row halo, owned rows per tile (ty == L: one full-height region, rows wrap)
  int ntx;          // tiles along x
  const int32_t *active;  // sample index per grid.y
  const uint4 *Esrc;      // [n][L][L/2] site pairs (P0, Q0, P1, Q1)
  const uint2 *Ssrc;      // [n][L/32][L/2] syndrome masks (s0, s1) of column pairs
  uint4 *Edst;
  uint2 *Sdst;
  uint32_t *alive;  // per sample: bit 0 anyons at pass start, bit j after step t_done+j
  uint32_t *wind;   // per sample winding bits: Wx(E), Wy(E), Wx(C), Wy(C)
  int *zero_count;  // counter to clear for the following compaction, or nullptr
  int m_max;        // limited-memory variant: 0 = no truncation
  int u;            // random moves every u steps, 0 = none
  const uint64_t *seeds;  // per sample: key of the random moves (read only when u > 0)
};

// Variant of a band-path batch: the limited-memory rule (see engine.h) or
// the open lattice.  Kernels are instantiated per mode (BAND_PLAIN,
// BAND_RULE, BAND_OPEN); the plain rule compiles without either.
enum BandMode { BAND_PLAIN = 0, BAND_RULE = 1, BAND_OPEN = 2 };
struct Rule {
  int m_max = 0;
  int u = 0;
  const uint64_t *seeds = nullptr;
  bool open = false;
  bool on() const { return m_max > 0 || u > 0; }
  int mode() const { return open ? BAND_OPEN : (on() ? BAND_RULE : BAND_PLAIN); }
};

// One pass of tile `tile` of `sample`, which has done t0 steps: loads the
// region from (Esrc, Ssrc), runs up to a.k steps, stores the owned part to
// (Edst, Sdst) (the Esrc/Ssrc/Edst/Sdst fields of `a` are not used).  A region has NW * 16
// rows.  With ty == L it spans the full height (L == NW * 16, rows wrap);
// otherwise regions overlap by hy rows (a multiple of 16) above and below.
// Returns, valid in thread 0: x = anyon bits of the owned part (bit 0 at the
// pass start, bit j after step j), y = winding bits of the correction links
// the pass flipped there.
//
// MODE BAND_OPEN: the open lattice (see k_resident): lanes and strips that
// lie outside [0, L) hold nothing, the rough-boundary columns 0 and L-1
// publish "emits now" in P and nothing in Q before every update (a boundary
// fold, run only by waves that hold such lanes), hold no anyon, and the
// full-height region (ty == L) reads a zero slot instead of its wrapped
// outer rows.  The correction winding is read on the x-links from column
// L-2 to L-1.
template <int NW, int MODE>
__device__ __forceinline__ uint2 band_region(const BandArgs &a, int tile, int sample, int t0, const uint4 *Esrc,
                                             const uint2 *Ssrc, uint4 *Edst, uint2 *Sdst) {
  constexpr bool RULE = MODE == BAND_RULE, OPEN = MODE == BAND_OPEN;
  extern __shared__ __align__(16) unsigned char smem[];
  uint4 *BND = reinterpret_cast<uint4 *>(smem);                         // [2][(NW+1)*2*64], slot NW stays 0
  uint2 *MB = reinterpret_cast<uint2 *>(BND + 2 * (NW + 1) * 2 * 64);  // [NW*64]
  uint32_t *red = reinterpret_cast<uint32_t *>(MB + NW * 64);      // [16]
  uint32_t *AW = red + 16;  // [16] per step of the pass: nonzero if anyons are left after it
  constexpr int H = BAND_H;
  constexpr uint32_t F = full_mask<H>();
  const int L = a.L;
  // Opaque thread index: in the kernels that run several regions per
  // workgroup, every lane-dependent value (columns, addresses, ownership) is
  // then formed anew per region instead of being kept live across the step
  // loop, whose register working set is close to the budget.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (scalar)
  const int ks = min(a.k, a.T_max - t0);  // steps of this sample in this pass
  if (threadIdx.x < 16) AW[threadIdx.x] = 0u;
  if (threadIdx.x == 0) red[0] = 0u;

  const bool wrapY = a.ty == L;
  const int tix = tile % a.ntx, tiy = tile / a.ntx;
  // neighbour strips (wrapped in a full-height region); for the message
  // updates the open full-height region reads the zero slot NW instead of
  // its wrapped outer rows (no move ever crosses those rows, so the move
  // exchange may keep the wrapped neighbours)
  const int wdn_f = w == 0 ? (wrapY ? NW - 1 : 0) : w - 1;
  const int wup_f = w == NW - 1 ? (wrapY ? 0 : NW - 1) : w + 1;
  const int wdn = (OPEN && wrapY && w == 0) ? NW : wdn_f;
  const int wup = (OPEN && wrapY && w == NW - 1) ? NW : wup_f;
  if (OPEN && threadIdx.x < 4 * 64) BND[(threadIdx.x >> 7) * (NW + 1) * 2 * 64 + NW * 2 * 64 + (threadIdx.x & 127)] =
      make_uint4(0u, 0u, 0u, 0u);
  // global column of this lane's first column, global row of the wave's first row
  const int tx0 = tix * a.tx, ty0 = tiy * a.ty;
  const int gx_raw = tx0 - a.hx + 2 * lane;
  int gx = gx_raw < 0 ? gx_raw + L : (gx_raw >= L ? gx_raw - L : gx_raw);
  const int gy_raw = (wrapY ? 0 : ty0 - a.hy) + w * H;
  int gy = gy_raw < 0 ? gy_raw + L : (gy_raw >= L ? gy_raw - L : gy_raw);
  // open lattice: lanes / strips outside the lattice, rough-boundary columns of this lane
  const bool outside = OPEN && (gx_raw < 0 || gx_raw >= L || gy_raw < 0 || gy_raw >= L);
  const bool bL = OPEN && gx_raw == 0, bR = OPEN && gx_raw == L - 2;
  const bool edge_wave = OPEN && __builtin_amdgcn_ballot_w64(outside || bL || bR) != 0ull;
  const int owned_w = min(a.tx, L - tx0);
  const bool own_col = 2 * lane >= a.hx && 2 * lane < a.hx + owned_w;
  // owned rows of this wave (wave-uniform); a strip never straddles row L-1 -> 0
  const int owned_h = wrapY ? L : min(a.ty, L - ty0);
  const int r0 = w * H - (wrapY ? 0 : a.hy);  // region row offset of the strip from the owned block
  uint32_t own_rows = 0u;
  if (r0 >= 0 && r0 + H <= owned_h) own_rows = F;
  else if (r0 + H > 0 && r0 < owned_h)
    for (int h = 0; h < H; ++h) own_rows |= (uint32_t)(r0 + h >= 0 && r0 + h < owned_h) << h;
  own_rows = __builtin_amdgcn_readfirstlane(own_rows);
  const bool own = own_col && own_rows != 0u;
  const bool top = !OPEN && gy == L - H && ((own_rows >> (H - 1)) & 1u);  // owns row L-1 (bit H-1)
  const bool last_col = own_col && gx == L - 2;  // torus: column L-1 is the second column; open: L-2 the first

  BandLane<H> b;
  uint32_t wind = 0u;
  const size_t half_row = (size_t)L / 2;
  const size_t sidx = ((size_t)sample * (L / TILE_H) + gy / TILE_H) * half_row + (gx >> 1);
  if (t0 == 0) {  // registers start empty; the syndrome comes from k_band_noise
#pragma unroll
    for (int h = 0; h < H; ++h) b.P0[h] = b.Q0[h] = b.P1[h] = b.Q1[h] = 0u;
  } else {
    const uint4 *E = Esrc + (size_t)sample * L * half_row;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const uint4 e = E[(size_t)(gy + h) * half_row + (gx >> 1)];
      b.P0[h] = e.x;
      b.Q0[h] = e.y;
      b.P1[h] = e.z;
      b.Q1[h] = e.w;
    }
  }
  {
    const uint2 sv = Ssrc[sidx];
    b.s0 = sv.x;
    b.s1 = sv.y;
  }
  if (OPEN) {  // nothing outside the lattice, no anyon on B
    if (outside) b.s0 = b.s1 = 0u;
    if (bL) b.s0 = 0u;
    if (bR) b.s1 = 0u;
  }

  const uint32_t own_mask = own_col ? own_rows : 0u;
  uint32_t bits = __syncthreads_or(((b.s0 | b.s1) & own_mask) != 0u) ? 1u : 0u;
  uint4 *BND0 = BND, *BND1 = BND + (NW + 1) * 2 * 64;
  uint32_t mk0 = 0u, mk1 = 0u;  // key of the random moves
  if (RULE && a.u > 0) {
    const uint64_t ms = a.seeds[sample];
    mk0 = (uint32_t)ms;
    mk1 = (uint32_t)(ms >> 32);
  }
  for (int st = 0; st < ks; ++st) {
    const uint32_t t3 = (uint32_t)(3 * (t0 + st));
    const uint32_t t1 = (uint32_t)(t0 + st + 1);  // the decoder step being applied
    const uint32_t rows = wave_rows<H>(b.s0, b.s1);
    Moves mv = {0u, 0u, 0u, 0u};
    // three message updates; LDS boundary slots alternate between sub-steps
    uint4 *slot_a = (st & 1) ? BND1 : BND0, *slot_b = (st & 1) ? BND0 : BND1;
    if (rows) band_fold<H>(b, (t3 + 1u) | ((t3 + 1u) << 16), rows);
    if (OPEN && edge_wave) band_boundary_fold<H>(b, (t3 + 1u) | ((t3 + 1u) << 16), outside, bL, bR);
    band_substep<H, false>(b, slot_a, w, wdn, wup, lane, rows, 1u, mv);
    if (rows) band_fold<H>(b, (t3 + 2u) | ((t3 + 2u) << 16), rows);
    if (OPEN && edge_wave) band_boundary_fold<H>(b, (t3 + 2u) | ((t3 + 2u) << 16), outside, bL, bR);
    band_substep<H, false>(b, slot_b, w, wdn, wup, lane, rows, 1u, mv);
    if (rows) band_fold<H>(b, (t3 + 3u) | ((t3 + 3u) << 16), rows);
    if (OPEN && edge_wave) band_boundary_fold<H>(b, (t3 + 3u) | ((t3 + 3u) << 16), outside, bL, bR);
    band_substep<H, true>(b, slot_a, w, wdn, wup, lane, rows, RULE ? live_threshold(t3 + 3u, a.m_max) : 1u, mv);
    if (RULE && a.u > 0 && t1 % (uint32_t)a.u == 0u) {  // random-move step (wave-uniform): replaces the decisions
      mv = {0u, 0u, 0u, 0u};
      band_random_moves<H>(b, rows, gx, gy, L, t1, mk0, mk1, mv);
    }
    uint32_t xo[2], yo[2];
    band_feedback<H>(b, mv, MB, w, wdn_f, wup_f, lane, xo, yo);
    if (OPEN) {  // anyons moved onto B are absorbed
      if (bL) b.s0 = 0u;
      if (bR) b.s1 = 0u;
      if (outside) b.s0 = b.s1 = 0u;
    }
    if (last_col) wind ^= (__popc(xo[OPEN ? 0 : 1] & own_rows) & 1u) << 2;
    if (own_col && top) wind ^= (((yo[0] ^ yo[1]) >> (H - 1)) & 1u) << 3;
    // anyons left after this step: waves OR into the step's flag, read after
    // the pass (no barrier of its own)
    const bool left = __ballot(((b.s0 | b.s1) & own_mask) != 0u) != 0ull;
    if (lane == 0 && left) atomicOr(&AW[st], 1u);
  }

  if (own && a.write_state) {
    uint4 *E = Edst + (size_t)sample * L * half_row;
#pragma unroll
    for (int h = 0; h < H; ++h)
      if ((own_rows >> h) & 1u)
        E[(size_t)(gy + h) * half_row + (gx >> 1)] = make_uint4(b.P0[h], b.Q0[h], b.P1[h], b.Q1[h]);
    // hy and ty are multiples of 16, so an owned strip is always whole
    Sdst[sidx] = make_uint2(b.s0, b.s1);
  }
  if (wind) atomicXor(&red[0], wind);
  __syncthreads();
  if (threadIdx.x == 0)
    for (int st = 0; st < ks; ++st) bits |= AW[st] ? 2u << st : 0u;
  return make_uint2(bits, red[0]);
}

// One pass over the samples in a.active: grid (tiles, samples).
template <int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void k_band(BandArgs a) {
  const int sample = a.active[blockIdx.y];
  if (a.zero_count != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.zero_count = 0;
  const int t0 = __builtin_amdgcn_readfirstlane(a.t_done[sample]);
  const uint2 r = band_region<NW, MODE>(a, blockIdx.x, sample, t0, a.Esrc, a.Ssrc, a.Edst, a.Sdst);
  if (threadIdx.x == 0) {
    if (r.x) atomicOr(&a.alive[sample], r.x);
    if (r.y) atomicXor(&a.wind[sample], r.y);
  }
}

// One pass over survivors whose number is only known on the device
// (*count): (sample, tile) tasks in a grid-stride loop, each as one k_band
// workgroup.  Workgroups never wait for each other.
template <int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void k_band_grid(BandArgs a, const int *count, int ntiles) {
  if (a.zero_count != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.zero_count = 0;
  const int64_t ntask = (int64_t)(*count) * ntiles;
  for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
    __syncthreads();  // the LDS slots of the previous task are no longer read
    const int i = (int)(task / ntiles), tile = (int)(task % ntiles);
    const int sample = a.active[i];
    const int t0 = __builtin_amdgcn_readfirstlane(a.t_done[sample]);
    const uint2 r = band_region<NW, MODE>(a, tile, sample, t0, a.Esrc, a.Ssrc, a.Edst, a.Sdst);
    if (threadIdx.x == 0) {
      if (r.x) atomicOr(&a.alive[sample], r.x);
      if (r.y) atomicXor(&a.wind[sample], r.y);
    }
  }
}

// Later passes of the band path, driven on the device.  Each workgroup takes
// the next surviving sample from `list` and runs its passes -- every tile of
// a pass one after another, then the bookkeeping of k_finalize for that
// sample -- until it is decoded or reaches T_max.  Workgroups share nothing
// but the atomic list head and never wait for each other; every one exits
// once the list is used up.
struct TailArgs {
  BandArgs a;  // tile geometry of a pass, k, T_max, wind
  int ntiles;
  int cur;     // buffer holding the survivors' state after the first pass
  uint4 *E[2];
  uint2 *S[2];
  const int32_t *list;  // survivors of the first pass
  const int *count;     // their number
  int *head;            // next list entry to take (zero before the launch)
  int32_t *t_done;
  int32_t *T_dec;
  uint8_t *status;
};

template <int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void k_band_tail(TailArgs ta) {
  __shared__ int s_take, s_more;
  __shared__ uint32_t s_bits, s_wind;
  const BandArgs &a = ta.a;
  const int nlist = *ta.count;
  for (;;) {
    __syncthreads();  // s_take of the previous sample has been read
    if (threadIdx.x == 0) s_take = atomicAdd(ta.head, 1);
    __syncthreads();
    const int i = __builtin_amdgcn_readfirstlane(s_take);
    if (i >= nlist) return;
    const int s = ta.list[i];
    int c = ta.cur;
    int t0 = __builtin_amdgcn_readfirstlane(ta.t_done[s]);
    for (;;) {
      const int ks = min(a.k, a.T_max - t0);  // >= 1: a survivor is below T_max
      if (threadIdx.x == 0) {
        s_bits = 1u;  // the sample held anyons when the pass started
        s_wind = 0u;
      }
      for (int tile = 0; tile < ta.ntiles; ++tile) {
        __syncthreads();  // the LDS slots of the previous tile are no longer read
        // buffers chosen by selects: an index into the kernel-argument arrays
        // would copy them to private memory
        const uint4 *Ein = c ? ta.E[1] : ta.E[0];
        uint4 *Eout = c ? ta.E[0] : ta.E[1];
        const uint2 *Sin = c ? ta.S[1] : ta.S[0];
        uint2 *Sout = c ? ta.S[0] : ta.S[1];
        const uint2 r = band_region<NW, MODE>(a, tile, s, t0, Ein, Sin, Eout, Sout);
        if (threadIdx.x == 0) {
          s_bits |= r.x;
          s_wind ^= r.y;
        }
      }
      // the state this pass stored is read by other waves in the next pass
      __threadfence();
      if (threadIdx.x == 0) {
        const uint32_t bits = s_bits;
        int td = -1;
        for (int j = 0; j <= ks; ++j)
          if (!((bits >> j) & 1u)) {
            td = t0 + j;
            break;
          }
        if (s_wind) a.wind[s] ^= s_wind;  // only this workgroup holds sample s
        ta.t_done[s] = t0 + ks;
        int more = 0;
        if (td >= 0) {
          ta.T_dec[s] = td;
          ta.status[s] = 1;
        } else if (t0 + ks >= a.T_max) {
          ta.T_dec[s] = a.T_max;
          ta.status[s] = (uint8_t)(2 | ((c ^ 1) << 2));
        } else {
          more = 1;
        }
        s_more = more;
      }
      __syncthreads();
      if (!s_more) break;
      t0 += ks;
      c ^= 1;
    }
  }
}

// Noise and initial syndrome of the band path, once per site.  A thread owns
// one column pair over one 16-row strip (the band's HBM word); a workgroup
// holds `CP` consecutive column pairs of `S` consecutive strips of one
// sample.  Writes the syndrome words and the error winding bits (Wx(E),
// Wy(E)) unless their pointers are null, and, if `counts` is set, the number
// of anyons in every 8x8 block as uint8 [n][L/8][L/8].  Links that cross into another workgroup (the y-links of
// the row below the group, the x-links left of its first column when the
// group is narrower than the lattice) are drawn again from the generator.
// With OPEN, links of the open lattice that do not exist are dropped (the
// x-links leaving column L-1, the y-links leaving row L-1 and those of the
// boundary columns 0 and L-1), the boundary columns carry no syndrome, and
// the error winding is read on the x-links from column L-2.
template <bool OPEN>
__global__ __launch_bounds__(1024) void k_band_noise(int L, int CP, int S, const uint64_t *seeds, uint64_t thr,
                                                     const double *p_arr, uint2 *Sout, uint32_t *wind,
                                                     uint8_t *counts) {
  constexpr bool open = OPEN;
  extern __shared__ __align__(16) unsigned char smem[];
  const int P = L / 2;                                  // column pairs of the lattice
  const int NB = CP / 4;                                // 8-column blocks of the group
  uint32_t *ex1s = reinterpret_cast<uint32_t *>(smem);  // [S][CP] x-links right of the second column
  uint32_t *eyts = ex1s + S * CP;                       // [S][CP] top-row y-links (bit 0 col 0, bit 1 col 1)
  uint32_t *cnt = eyts + S * CP;                        // [2S][NB] anyon counts of the group's blocks
  uint32_t *red = cnt + 2 * S * NB;
  const int gxn = P / CP, gyn = (L / TILE_H) / S;
  const int64_t sample = blockIdx.x / (gxn * gyn);
  const int grp = (int)(blockIdx.x % (gxn * gyn));
  const int cx = grp % gxn, cy = grp / gxn;
  const int tid = threadIdx.x, ql = tid % CP, jl = tid / CP;
  const int q = cx * CP + ql, j = cy * S + jl, y0 = j * TILE_H, gx = 2 * q;
  for (int i = tid; i < 2 * S * NB; i += blockDim.x) cnt[i] = 0u;
  if (tid == 0) red[0] = 0u;
  const uint64_t seed = seeds[sample];
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint64_t t = p_arr ? device_threshold(p_arr[sample]) : thr;
  // rows from the top down, each flip bit shifted in at bit 0 through the
  // carry of one add (shift_in_below), so row h ends at bit h; t = 2^32
  // (p = 1) flips every link, below that the 32-bit comparison is exact
  const uint32_t t32 = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
  uint32_t ex0 = 0u, ey0 = 0u, ex1 = 0u, ey1 = 0u;
#pragma unroll 4
  for (int h = TILE_H - 1; h >= 0; --h) {
    const Words4 r = philox4x32_10((uint32_t)((y0 + h) * L + gx) >> 1, k0, k1);
    shift_in_below(ex0, r.w0, t32);
    shift_in_below(ey0, r.w1, t32);
    shift_in_below(ex1, r.w2, t32);
    shift_in_below(ey1, r.w3, t32);
  }
  if (t > 0xFFFFFFFFull) ex0 = ey0 = ex1 = ey1 = full_mask<TILE_H>();
  if (open) {
    if (q == P - 1) ex1 = 0u;                       // x-links leaving column L-1
    if (q == 0) ey0 = 0u;                           // column 0 is the boundary
    if (q == P - 1) ey1 = 0u;                       // column L-1 is the boundary
    if (y0 + TILE_H == L) {                         // y-links leaving row L-1
      ey0 &= ~(1u << (TILE_H - 1));
      ey1 &= ~(1u << (TILE_H - 1));
    }
  }
  uint32_t eyd = 0u;  // y-links of the row below the strip (bit 0 col 0, bit 1 col 1)
  if (jl == 0 && !(open && y0 == 0)) {  // that row belongs to another workgroup
    const int yb = y0 == 0 ? L - 1 : y0 - 1;
    const Words4 r = philox4x32_10((uint32_t)(yb * L + gx) >> 1, k0, k1);
    eyd = (uint32_t)((uint64_t)r.w1 < t) | ((uint32_t)((uint64_t)r.w3 < t) << 1);
    if (open) eyd &= (q == 0 ? 2u : 3u) & (q == P - 1 ? 1u : 3u);
  }
  uint32_t exl = 0u;  // x-links entering column 2q from the left
  if (ql == 0 && CP < P && !(open && q == 0)) {
    const int xl = gx == 0 ? L - 2 : gx - 2;  // pair holding column 2q-1 as its second column
#pragma unroll 4
    for (int h = 0; h < TILE_H; ++h) {
      const Words4 r = philox4x32_10((uint32_t)((y0 + h) * L + xl) >> 1, k0, k1);
      exl |= (uint32_t)((uint64_t)r.w2 < t) << h;
    }
  }
  ex1s[jl * CP + ql] = ex1;
  eyts[jl * CP + ql] = ((ey0 >> (TILE_H - 1)) & 1u) | (((ey1 >> (TILE_H - 1)) & 1u) << 1);
  __syncthreads();
  if (ql > 0 || CP == P) exl = ex1s[jl * CP + (ql == 0 ? CP - 1 : ql - 1)];
  if (jl > 0) eyd = eyts[(jl - 1) * CP + ql];
  constexpr uint32_t F = full_mask<TILE_H>();
  uint32_t s0 = (ex0 ^ exl ^ ey0 ^ ((ey0 << 1) | (eyd & 1u))) & F;
  uint32_t s1 = (ex1 ^ ex0 ^ ey1 ^ ((ey1 << 1) | (eyd >> 1))) & F;
  if (open) {  // the boundary columns carry no syndrome
    if (q == 0) s0 = 0u;
    if (q == P - 1) s1 = 0u;
  }
  if (Sout != nullptr) Sout[((size_t)sample * (L / TILE_H) + j) * P + q] = make_uint2(s0, s1);
  uint32_t wd = 0u;
  if (open) {
    if (q == P - 1) wd ^= __popc(ex0) & 1u;  // x-links from column L-2 to L-1
  } else {
    if (q == P - 1) wd ^= __popc(ex1) & 1u;                                  // x-links leaving column L-1
    if (j == L / TILE_H - 1) wd ^= (((ey0 ^ ey1) >> (TILE_H - 1)) & 1u) << 1;  // y-links leaving row L-1
  }
  if (wd) atomicXor(&red[0], wd);
  if (counts != nullptr) {
    const int bx = ql / 4;  // 8 columns = 4 pairs per block
    atomicAdd(&cnt[(2 * jl) * NB + bx], __popc(s0 & 0xFFu) + __popc(s1 & 0xFFu));
    atomicAdd(&cnt[(2 * jl + 1) * NB + bx], __popc(s0 >> 8) + __popc(s1 >> 8));
  }
  __syncthreads();
  if (wind != nullptr && tid == 0 && red[0]) atomicXor(&wind[sample], red[0]);
  if (counts != nullptr) {
    uint8_t *out = counts + (size_t)sample * (L / 8) * (L / 8) + (size_t)(2 * cy * S) * (L / 8) + cx * NB;
    for (int i = tid; i < 2 * S * NB; i += blockDim.x) out[(i / NB) * (L / 8) + i % NB] = (uint8_t)cnt[i];
  }
}

// Per-pass bookkeeping: T_dec from the per-step bits, compaction of the
// samples that still hold anyons.  The pass covered active[0 .. nact) or, if
// nact_dev is set, active[0 .. *nact_dev) (nact is then an upper bound).  status: 0 running, 1 decoded, 2 timeout;
// bit 2 of a timeout: the state buffer (0/1) that holds its final syndrome
// (samples of first-pass groups of different depth time out in different
// passes).  `dst` is the buffer this pass wrote.
__global__ void k_finalize(int k, int T_max, int dst, const int32_t *active, int nact, const int *nact_dev,
                           int32_t *t_done, uint32_t *alive, int32_t *T_dec, uint8_t *status, int32_t *next,
                           int *next_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (nact_dev != nullptr ? *nact_dev : nact)) return;
  const int s = active[i];
  const int t0 = t_done[s];
  const int ks = min(k, T_max - t0);
  const uint32_t bits = alive[s] | (t0 == 0 ? 0u : 1u);
  alive[s] = 0u;
  t_done[s] = t0 + ks;
  int td = -1;
  for (int j = 0; j <= ks; ++j)
    if (!((bits >> j) & 1u)) {
      td = t0 + j;
      break;
    }
  if (td >= 0) {
    T_dec[s] = td;
    status[s] = 1;
  } else if (t0 + ks >= T_max) {
    T_dec[s] = T_max;
    status[s] = (uint8_t)(2 | (dst << 2));
  } else {
    next[atomicAdd(next_count, 1)] = s;
  }
}

__global__ void k_tile_init(int64_t n, uint32_t *alive, uint32_t *wind, uint8_t *status, int32_t *t_done,
                            int32_t *active, int *tail_head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == 0) *tail_head = 0;
  alive[i] = 0u;
  wind[i] = 0u;
  status[i] = 0;
  t_done[i] = 0;
  active[i] = (int32_t)i;
}

// flags and final syndrome (row-major bits) from the band state.
__global__ void k_band_export(int L, int64_t n, const uint8_t *status, const uint32_t *wind,
                              const uint2 *S0, const uint2 *S1, uint8_t *flags, uint32_t *syn) {
  const int64_t smp = blockIdx.x;
  const int64_t nw = ((int64_t)L * L + 31) / 32;
  const bool timeout = (status[smp] & 3) == 2;
  const uint2 *Slast = (status[smp] >> 2) & 1 ? S1 : S0;
  if (threadIdx.x == 0) {
    const uint32_t W = wind[smp];
    const uint32_t fail = ((W ^ (W >> 2)) & 3u) != 0u;
    flags[smp] = (uint8_t)((fail | (timeout ? 1u : 0u)) | (timeout ? 2u : 0u));
  }
  if (syn == nullptr) return;
  const size_t half_row = (size_t)L / 2;
  for (int64_t wd = threadIdx.x; wd < nw; wd += blockDim.x) {
    uint32_t word = 0u;
    if (timeout) {
      for (int bt = 0; bt < 32; ++bt) {
        const int64_t i = wd * 32 + bt;
        const int y = (int)(i / L), x = (int)(i % L);
        const uint2 m = Slast[((size_t)smp * (L / TILE_H) + y / TILE_H) * half_row + (x >> 1)];
        word |= (((x & 1) ? m.y : m.x) >> (y % TILE_H) & 1u) << bt;
      }
    }
    syn[smp * nw + wd] = word;
  }
}

// ---------------------------------------------------------------------------
// Band path: explicit errors and the full state (checkpoint / resume)
// ---------------------------------------------------------------------------

// Initial syndrome and error winding of explicit error patterns in the band
// layout (instead of k_band_noise).  One thread per sample, 16-row strip j
// and column pair q.  Link id 2i + dir of site i = y L + x puts the four
// links of the pair (x-link 2q, y-link 2q, x-link 2q+1, y-link 2q+1) of row y
// in the nibble (y L/2 + q) of the sample's link words.
__global__ void k_band_links(int L, int64_t n, const uint32_t *links, uint2 *Sout, uint32_t *wind) {
  const int P = L / 2, NJ = L / TILE_H;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * NJ * P) return;
  const int64_t sample = g / ((int64_t)NJ * P);
  const int j = (int)((g / P) % NJ), q = (int)(g % P);
  const uint32_t *w = links + sample * ((int64_t)L * L / 16);
  auto nib = [&](int y, int qq) -> uint32_t {
    const size_t idx = (size_t)y * P + qq;
    return (w[idx >> 3] >> ((idx & 7u) * 4u)) & 0xFu;
  };
  const int ql = q == 0 ? P - 1 : q - 1;
  uint32_t s0 = 0u, s1 = 0u, wd = 0u;
  for (int h = 0; h < TILE_H; ++h) {
    const int y = j * TILE_H + h, yd = y == 0 ? L - 1 : y - 1;
    const uint32_t c = nib(y, q), l = nib(y, ql), d = nib(yd, q);
    // sigma = ex ^ ex(left) ^ ey ^ ey(below)
    s0 |= (((c >> 0) ^ (l >> 2) ^ (c >> 1) ^ (d >> 1)) & 1u) << h;
    s1 |= (((c >> 2) ^ (c >> 0) ^ (c >> 3) ^ (d >> 3)) & 1u) << h;
    if (q == P - 1) wd ^= (c >> 2) & 1u;                            // x-links leaving column L-1
    if (y == L - 1) wd ^= (((c >> 1) ^ (c >> 3)) & 1u) << 1;        // y-links leaving row L-1
  }
  Sout[((size_t)sample * NJ + j) * P + q] = make_uint2(s0, s1);
  if (wd) atomicXor(&wind[sample], wd);
}

// Steps done after a pass of k steps with no early exit (every sample runs
// to t_end); the per-step anyon bits are not needed.
__global__ void k_band_advance(int64_t n, int k, int t_end, int32_t *t_done, uint32_t *alive) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  t_done[s] = min(t_done[s] + k, t_end);
  alive[s] = 0u;
}

// Exported state (registers [n][4][L L] int16 in distance form, syndrome
// bits, winding bits) after t0 steps -> band layout with emission times
// e = 3 t0 - m + 1 (0 for m = 0).  One thread per sample, strip and pair.
__global__ void k_band_state_import(int L, int64_t n, int t0, const int16_t *m_in, const uint32_t *syn_in,
                                    const uint8_t *wind_in, uint4 *E, uint2 *S, uint32_t *wind, int32_t *t_done) {
  const int P = L / 2, NJ = L / TILE_H;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * NJ * P) return;
  const int64_t sample = g / ((int64_t)NJ * P);
  const int j = (int)((g / P) % NJ), q = (int)(g % P);
  const int64_t n2 = (int64_t)L * L, nw = n2 / 32;
  const int16_t *mi = m_in + sample * 4 * n2;
  const uint32_t s0t = 3u * (uint32_t)t0;
  auto em = [&](int d, int64_t i) -> uint32_t {
    const uint32_t m = (uint32_t)(uint16_t)mi[d * n2 + i];
    return m != 0u ? ((s0t - m + 1u) & 0xFFFFu) : 0u;
  };
  uint32_t s0 = 0u, s1 = 0u;
  for (int h = 0; h < TILE_H; ++h) {
    const int y = j * TILE_H + h;
    const int64_t i = (int64_t)y * L + 2 * q;
    E[(size_t)sample * L * P + (size_t)y * P + q] =
        make_uint4(em(0, i) | em(1, i) << 16, em(2, i) | em(3, i) << 16, em(0, i + 1) | em(1, i + 1) << 16,
                   em(2, i + 1) | em(3, i + 1) << 16);
    const uint32_t word = syn_in[sample * nw + (i >> 5)];
    s0 |= ((word >> (i & 31)) & 1u) << h;
    s1 |= ((word >> ((i + 1) & 31)) & 1u) << h;
  }
  S[((size_t)sample * NJ + j) * P + q] = make_uint2(s0, s1);
  if (j == 0 && q == 0) {
    wind[sample] = wind_in[sample] & 15u;
    t_done[sample] = t0;
  }
}

// Band state after `steps` steps -> exported form: registers in distance
// form m = s - e + 1 for live emission times (s = 3 steps; none before the
// first step), syndrome bits row-major, winding bits.  Grid: one thread per
// sample and syndrome word.
__global__ void k_band_state_export(int L, int64_t n, int steps, int m_max, const uint4 *E, const uint2 *S,
                                    const uint32_t *wind, int16_t *m_out, uint32_t *syn_out, uint8_t *wind_out) {
  const int P = L / 2, NJ = L / TILE_H;
  const int64_t n2 = (int64_t)L * L, nw = n2 / 32;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * nw) return;
  const int64_t sample = g / nw, wd = g % nw;
  const uint32_t snow = 3u * (uint32_t)steps;
  const uint32_t live = live_threshold(snow, m_max);
  int16_t *mo = m_out + sample * 4 * n2;
  uint32_t word = 0u;
  for (int bt = 0; bt < 32; bt += 2) {
    const int64_t i = wd * 32 + bt;
    const int y = (int)(i / L), x = (int)(i % L), q = x >> 1;
    const uint2 sv = S[((size_t)sample * NJ + y / TILE_H) * P + q];
    word |= ((sv.x >> (y % TILE_H)) & 1u) << bt;
    word |= ((sv.y >> (y % TILE_H)) & 1u) << (bt + 1);
    uint4 e = make_uint4(0u, 0u, 0u, 0u);
    if (steps > 0) e = E[(size_t)sample * L * P + (size_t)y * P + q];
    const uint32_t v[8] = {e.x & 0xFFFFu, e.x >> 16, e.y & 0xFFFFu, e.y >> 16,
                           e.z & 0xFFFFu, e.z >> 16, e.w & 0xFFFFu, e.w >> 16};
    for (int c = 0; c < 2; ++c)
      for (int d = 0; d < 4; ++d) {
        const uint32_t ev = v[4 * c + d];
        mo[d * n2 + i + c] = (int16_t)(steps > 0 && ev >= live ? (snow - ev + 1u) : 0u);
      }
  }
  syn_out[sample * nw + wd] = word;
  if (wd == 0) wind_out[sample] = (uint8_t)(wind[sample] & 15u);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

thread_local std::string g_last_error;

int fail_with(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

Profiler g_prof;

int cu_count() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  return cache[dev] = cus;
}

uint64_t threshold_of(double p) {
  double t = floor(p * 4294967296.0);
  if (t < 0.0) t = 0.0;
  if (t > 4294967296.0) t = 4294967296.0;
  return (uint64_t)t;
}

// Strip height for the resident kernel: the divisor H <= 16 of L giving the
// block size L*L/H closest to 256 threads without exceeding 1024.
int resident_H(int L) {
  // Measured on MI355X (4096 samples per batch): where the rule below picks
  // H = 16 the strips spill registers, and these heights decode faster at
  // p = 0.01 -- L = 64: 1.7x, 80: 1.5x, 96: 1.9x, 112: 1.5x.  At other sizes
  // a sweep of every height at p = 0.01 and 0.03 found these faster than the
  // rule's -- L = 24: 1.1-1.3x, 40: 1.06x, 48: 1.75x, 60: 1.27x.
  if (L == 24) return 3;
  if (L == 40) return 5;
  if (L == 48) return 12;
  if (L == 60) return 5;
  if (L == 64) return 8;
  if (L == 80) return 10;
  if (L == 96) return 12;
  if (L == 112) return 14;
  // The divisor H <= 16 of L giving the block size closest to 256 threads
  // without exceeding 1024.
  int best = 0;
  long bestd = 1L << 40;
  for (int H = 1; H <= 16; ++H) {
    if (L % H) continue;
    const long th = (long)L * L / H;
    if (th > 1024) continue;
    const long d = th > 256 ? th - 256 : 256 - th;
    if (d < bestd) {
      bestd = d;
      best = H;
    }
  }
  return best;
}

// Region rows, the move/link exchange and the reduction word; one more row
// (the zero row) for the open lattice.
size_t resident_lds(int L, int H, bool open = false) {
  return (size_t)L * (open ? L + 1 : L) * sizeof(uint2) + (size_t)L * (L / H) * sizeof(uint4) + 64;
}

size_t band_lds(int nw) {  // boundary slots of nw strips plus a zero slot, move masks, flags
  return (size_t)2 * (nw + 1) * 2 * 64 * sizeof(uint4) + (size_t)nw * 64 * sizeof(uint2) + 64 + 64;
}

template <int H>
int launch_resident_h(const ResidentArgs &a, hipStream_t stream) {
  const size_t lds = resident_lds(a.L, H, a.open != 0);
  const int threads = a.L * a.L / H;
  ProfScope ps("k_resident", stream);
  if (a.open)
    hipLaunchKernelGGL((k_resident<H, RES_OPEN>), dim3((unsigned)a.n), dim3(threads), lds, stream, a);
  else if (a.m_max > 0 || a.u > 0)
    hipLaunchKernelGGL((k_resident<H, RES_RULE>), dim3((unsigned)a.n), dim3(threads), lds, stream, a);
  else
    hipLaunchKernelGGL((k_resident<H, RES_PLAIN>), dim3((unsigned)a.n), dim3(threads), lds, stream, a);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

int launch_resident(const ResidentArgs &a, hipStream_t stream) {
  switch (resident_H(a.L)) {
    case 1: return launch_resident_h<1>(a, stream);
    case 2: return launch_resident_h<2>(a, stream);
    case 3: return launch_resident_h<3>(a, stream);
    case 4: return launch_resident_h<4>(a, stream);
    case 5: return launch_resident_h<5>(a, stream);
    case 6: return launch_resident_h<6>(a, stream);
    case 7: return launch_resident_h<7>(a, stream);
    case 8: return launch_resident_h<8>(a, stream);
    case 9: return launch_resident_h<9>(a, stream);
    case 10: return launch_resident_h<10>(a, stream);
    case 11: return launch_resident_h<11>(a, stream);
    case 12: return launch_resident_h<12>(a, stream);
    case 13: return launch_resident_h<13>(a, stream);
    case 14: return launch_resident_h<14>(a, stream);
    case 15: return launch_resident_h<15>(a, stream);
    case 16: return launch_resident_h<16>(a, stream);
    default: return fail_with(MPD_ERR_L, "L=%d has no strip height for the resident kernel", a.L);
  }
}

// The whole-lattice band kernel takes seeded plain-rule decodes at L = 64
// (one column per lane, 4 waves) and L = 128 (two columns per lane, 8
// waves); every other small lattice, explicit errors, state export and the
// rule variants use k_resident.
bool torus_ok(int L) { return L == 64 || L == 128; }

// Workgroups of k_torus that fit on the device at once (CUs x occupancy).
int torus_resident_groups(const void *kernel, int threads, size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess)
    return 0;
  return std::max(cus * per_cu, 0);
}

// resident_grid: the launch resumes a batch of which the bit-sliced kernel
// is expected to have decoded nearly every sample, so one grid of resident
// workgroups steps over it instead of a workgroup per sample.  A fixed share
// of samples per workgroup balances badly once many are left (decode times
// have a long tail near the threshold), so every other launch leaves the
// balancing to the hardware, one workgroup per sample.
int launch_torus(int L, const TorusArgs &a, bool resident_grid, hipStream_t stream) {
  ProfScope ps("k_torus", stream);
  if (L == 64) {
    const size_t lds = (size_t)2 * 4 * 2 * 64 * sizeof(uint2) + (size_t)4 * 64 * sizeof(uint2);
    static const int cap64 = torus_resident_groups((const void *)k_torus<1, 4>, 4 * 64, lds);
    const int64_t g = a.resume && resident_grid && cap64 > 0 ? std::min<int64_t>(a.n, cap64) : a.n;
    hipLaunchKernelGGL((k_torus<1, 4>), dim3((unsigned)g), dim3(4 * 64), lds, stream, a);
  } else {
    const size_t lds = (size_t)2 * 8 * 2 * 64 * sizeof(uint4) + (size_t)8 * 64 * sizeof(uint2);
    static const int cap128 = torus_resident_groups((const void *)k_torus<2, 8>, 8 * 64, lds);
    const int64_t g = a.resume && resident_grid && cap128 > 0 ? std::min<int64_t>(a.n, cap128) : a.n;
    hipLaunchKernelGGL((k_torus<2, 8>), dim3((unsigned)g), dim3(8 * 64), lds, stream, a);
  }
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

int bits_steps_for(int L);  // bit-sliced steps of the schedule for L (below)

// A seeded plain-rule decode of a small lattice (one workgroup per sample):
// the whole-lattice band kernel where it applies, else the resident kernel.
int launch_small(int L, int64_t n, const uint64_t *seeds, uint64_t thr, const double *p_arr, int T_max,
                 int32_t *T_dec, uint8_t *flags, uint32_t *syn, hipStream_t stream) {
  if (torus_ok(L)) {
    TorusArgs t;
    t.n = n;
    t.seeds = seeds;
    t.thr = thr;
    t.p_arr = p_arr;
    t.T_max = T_max;
    t.T_dec = T_dec;
    t.flags = flags;
    t.syn = syn;
    // With one p for the batch (p_arr null), the share of samples left after
    // the bit-sliced steps follows from p.  Measured at L = 64 (10000
    // samples) and 128 (4096): up to p = 0.02 so few are left that a
    // resident grid resumes them fastest; from p = 0.045 on nearly every
    // sample is left, and the bit-sliced steps only add their own time to a
    // decode the whole-lattice kernel does again, so they are skipped.
    // Per-sample p keeps the steps and resumes one workgroup per sample.
    const bool one_p = p_arr == nullptr;
    const int kb_set = one_p && thr >= threshold_of(0.045) ? 0 : bits_steps_for(L), kb = std::min(kb_set, T_max);
    if (kb_set > 0) {
      // noise and the first kb steps bit-sliced; the whole-lattice kernel
      // takes the samples that are still decoding after them
      BitsArgs b = {};
      b.seeds = seeds;
      b.thr = thr;
      b.p_arr = p_arr;
      b.k = kb;
      b.T_max = T_max;
      b.T_dec = T_dec;
      b.flags = flags;
      b.syn = syn;
      {
        ProfScope ps("k_bits_small", stream);
        if (L == 64)
          hipLaunchKernelGGL((k_bits<false, 1>), dim3((unsigned)n), dim3(64), 0, stream, b);
        else
          hipLaunchKernelGGL((k_bits<false, 2>), dim3((unsigned)n), dim3(128), 0, stream, b);
      }
      HIP_TRY(hipGetLastError());
      if (T_max <= kb) return MPD_OK;
      t.resume = 1;
    }
    return launch_torus(L, t, one_p && thr <= threshold_of(0.02), stream);
  }
  ResidentArgs a = {};
  a.L = L;
  a.n = n;
  a.seeds = seeds;
  a.thr = thr;
  a.p_arr = p_arr;
  a.links = nullptr;
  a.T_max = T_max;
  a.t_exact = -1;
  a.T_dec = T_dec;
  a.flags = flags;
  a.syn = syn;
  return launch_resident(a, stream);
}

bool resident_ok(int L) {
  if (L < 3 || L > 128) return false;
  const int H = resident_H(L);
  return H > 0 && resident_lds(L, H) <= 160 * 1024;
}

// The band path: L = 256 (one full-height region) or larger multiples of 16.
bool tiled_ok(int L) { return L >= BAND_RY && L % TILE_H == 0 && L <= 16384; }

struct BandWorkspace {
  uint4 *E[2];      // [n][L][L/2] register pairs
  uint2 *S[2];      // [n][L/32][L/2] syndrome masks of column pairs
  uint32_t *alive, *wind;
  uint8_t *status;
  int32_t *t_done;
  int32_t *active[2];
  int *count;  // [3]: survivors after passes into buffer 0 / 1; list head of the device-driven passes
  size_t bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

BandWorkspace band_layout(int L, int64_t n, void *base) {
  BandWorkspace w;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void *p = base ? (void *)((char *)base + off) : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t sites = (size_t)n * L * L;
  for (int b = 0; b < 2; ++b) w.E[b] = (uint4 *)take(sites * sizeof(uint2));
  for (int b = 0; b < 2; ++b) w.S[b] = (uint2 *)take((size_t)n * (L / TILE_H) * (L / 2) * sizeof(uint2));
  w.alive = (uint32_t *)take((size_t)n * 4);
  w.wind = (uint32_t *)take((size_t)n * 4);
  w.status = (uint8_t *)take((size_t)n);
  w.t_done = (int32_t *)take((size_t)n * 4);
  for (int b = 0; b < 2; ++b) w.active[b] = (int32_t *)take((size_t)n * 4);
  w.count = (int *)take(3 * sizeof(int));
  w.bytes = off;
  return w;
}

// Decoder steps per pass (first pass, later passes).  With 128-column
// regions a halo of 4k leaves 128 - 8k owned columns per tile: L = 256
// takes 3 tiles for k <= 5.
struct BandSchedule {
  int k_first = 4;
  int k_next = 2;
  int driver = MPD_BAND_DRIVER_AUTO;
  int k_bits = BITS_MAX_STEPS;  // steps of the bit-sliced first kernel (L = 256, plain rule); 0 = band first pass
};
std::mutex g_sched_mu;
BandSchedule g_sched_default;
std::map<int, BandSchedule> g_sched_by_L;  // set by the autotuner or the caller

BandSchedule schedule_for(int L) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  auto it = g_sched_by_L.find(L);
  return it == g_sched_by_L.end() ? g_sched_default : it->second;
}
int bits_steps_for(int L) { return schedule_for(L).k_bits; }

// Launch shape of k_band_noise: whole rows of column pairs when they fit in
// one workgroup, else the widest divisor of L/2 (a multiple of 4, so that
// 8x8 blocks stay inside a group); then as many strips as fit.
struct NoiseShape {
  int CP, S, groups;
  size_t lds;
};
NoiseShape noise_shape(int L) {
  NoiseShape g;
  const int P = L / 2;
  g.CP = P;
  if (P > 1024)
    for (g.CP = 1024; g.CP > 4 && (P % g.CP || g.CP % 4); --g.CP) {
    }
  g.S = 1024 / g.CP;
  while (g.S > 1 && (L / TILE_H) % g.S) --g.S;
  g.groups = (P / g.CP) * ((L / TILE_H) / g.S);
  g.lds = (size_t)(2 * g.S * g.CP + 2 * g.S * (g.CP / 4) + 4) * sizeof(uint32_t);
  return g;
}

// Noise, syndrome and bookkeeping of a band-path batch (before the passes).
int band_start(int L, uint64_t thr, const double *d_p, const uint64_t *d_seeds, int64_t n, const BandWorkspace &w,
               uint8_t *d_counts, hipStream_t stream, int open = 0, const uint32_t *d_links = nullptr) {
  hipLaunchKernelGGL(k_tile_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, w.alive, w.wind,
                     w.status, w.t_done, w.active[0], &w.count[2]);
  HIP_TRY(hipGetLastError());
  if (d_links != nullptr) {  // explicit error patterns instead of seeded noise
    const int64_t threads = n * (L / TILE_H) * (L / 2);
    hipLaunchKernelGGL(k_band_links, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, L, n, d_links,
                       w.S[0], w.wind);
    HIP_TRY(hipGetLastError());
    return MPD_OK;
  }
  const NoiseShape g = noise_shape(L);
  ProfScope ps("k_band_noise", stream);
  if (open)
    hipLaunchKernelGGL(k_band_noise<true>, dim3((unsigned)(n * g.groups)), dim3(g.CP * g.S), g.lds, stream, L, g.CP,
                       g.S, d_seeds, thr, d_p, w.S[0], w.wind, d_counts);
  else
    hipLaunchKernelGGL(k_band_noise<false>, dim3((unsigned)(n * g.groups)), dim3(g.CP * g.S), g.lds, stream, L, g.CP,
                       g.S, d_seeds, thr, d_p, w.S[0], w.wind, d_counts);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

// One pass of up to k steps over the samples in `active` (state in buffers
// cur, written to cur ^ 1), then T_dec bookkeeping and compaction of the
// survivors into w.active[cur ^ 1].  `zero` clears the survivor counter
// first (the first launch of a pass).
// Would a pass of k steps over nact samples in full-size regions leave
// compute units idle?
bool small_pass(int L, int k, int nact) {
  const int tx = BAND_RX - 8 * k;
  const int hy = (4 * k + TILE_H - 1) / TILE_H * TILE_H;
  const int ty16 = L == BAND_RY ? L : BAND_RY - 2 * hy;
  const int64_t wg16 = (int64_t)((L + tx - 1) / tx) * ((L + ty16 - 1) / ty16) * nact;
  return wg16 < cu_count();
}

// Steps of a later pass: the schedule's k_next, but at least K_SMALL when the
// pass is small -- it then runs in 4-wave regions at a fraction of the time
// per step, and a round trip to the host costs more than a few extra steps.
constexpr int K_SMALL = 4;
int later_pass_k(int L, int nact) {
  const int kn = schedule_for(L).k_next;
  return (kn < K_SMALL && small_pass(L, kn, nact)) ? K_SMALL : kn;
}

// Tiles of a pass of k steps in regions of ry rows: a halo of 4k columns and
// of 4k rows rounded up to whole 16-row strips (none when one region spans
// the height).  Fills the geometry fields of `ba`; returns the tiles along y.
int tile_geometry(int L, int k, int ry, BandArgs &ba) {
  ba.L = L;
  ba.write_state = 1;
  ba.k = k;
  ba.hx = 4 * k;
  ba.tx = BAND_RX - 2 * ba.hx;
  ba.ntx = (L + ba.tx - 1) / ba.tx;
  const int hy = (4 * k + TILE_H - 1) / TILE_H * TILE_H;
  if (L == ry) {
    ba.hy = 0;
    ba.ty = L;
  } else {
    ba.hy = hy;
    ba.ty = ry - 2 * hy;
  }
  return (L + ba.ty - 1) / ba.ty;
}

int band_pass(int L, int k, int T_max, const BandWorkspace &w, const int32_t *active, int nact, int cur, bool zero,
              int32_t *d_T_dec, const Rule &rule, hipStream_t stream) {
  BandArgs ba;
  // Full-size regions (16 waves, 256 rows) unless their grid would leave
  // compute units idle: then 4-wave regions of 64 rows, which need more
  // (overlapping) tiles but take about a quarter of the time per step.
  const int hy = (4 * k + TILE_H - 1) / TILE_H * TILE_H;
  const int ry4 = BAND_NW_SMALL * BAND_H;
  const bool small = small_pass(L, k, nact) && ry4 - 2 * hy >= TILE_H;
  const int nty = tile_geometry(L, k, small ? ry4 : BAND_RY, ba);
  ba.T_max = T_max;
  ba.t_done = w.t_done;
  ba.active = active;
  ba.Esrc = w.E[cur];
  ba.Ssrc = w.S[cur];
  ba.Edst = w.E[cur ^ 1];
  ba.Sdst = w.S[cur ^ 1];
  ba.alive = w.alive;
  ba.wind = w.wind;
  ba.zero_count = zero ? &w.count[cur ^ 1] : nullptr;
  ba.m_max = rule.m_max;
  ba.u = rule.u;
  ba.seeds = rule.seeds;
  {
    ProfScope ps("k_band", stream);
    const dim3 grid((unsigned)(ba.ntx * nty), (unsigned)nact);
    if (small) {
      const dim3 blk(BAND_NW_SMALL * 64);
      const size_t lds = band_lds(BAND_NW_SMALL);
      switch (rule.mode()) {
        case BAND_RULE: hipLaunchKernelGGL((k_band<BAND_NW_SMALL, BAND_RULE>), grid, blk, lds, stream, ba); break;
        case BAND_OPEN: hipLaunchKernelGGL((k_band<BAND_NW_SMALL, BAND_OPEN>), grid, blk, lds, stream, ba); break;
        default: hipLaunchKernelGGL((k_band<BAND_NW_SMALL, BAND_PLAIN>), grid, blk, lds, stream, ba);
      }
    } else {
      const dim3 blk(BAND_NW * 64);
      const size_t lds = band_lds(BAND_NW);
      switch (rule.mode()) {
        case BAND_RULE: hipLaunchKernelGGL((k_band<BAND_NW, BAND_RULE>), grid, blk, lds, stream, ba); break;
        case BAND_OPEN: hipLaunchKernelGGL((k_band<BAND_NW, BAND_OPEN>), grid, blk, lds, stream, ba); break;
        default: hipLaunchKernelGGL((k_band<BAND_NW, BAND_PLAIN>), grid, blk, lds, stream, ba);
      }
    }
  }
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((nact + 255) / 256)), dim3(256), 0, stream, k, T_max, cur ^ 1, active,
                     nact, (const int *)nullptr, w.t_done, w.alive, d_T_dec, w.status, w.active[cur ^ 1],
                     &w.count[cur ^ 1]);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

// A pass like band_pass over a list whose length is only known on the
// device (*count, at most `bound`): the persistent k_band_grid walks the
// (sample, tile) tasks and k_finalize reads the count itself, so the host
// does not wait for it.
int band_pass_dev(int L, int k, int T_max, const BandWorkspace &w, const int32_t *active, const int *count,
                  int64_t bound, int cur, bool zero, int32_t *d_T_dec, const Rule &rule, hipStream_t stream) {
  BandArgs ba;
  const int nty = tile_geometry(L, k, BAND_RY, ba);
  const int ntiles = ba.ntx * nty;
  ba.T_max = T_max;
  ba.t_done = w.t_done;
  ba.active = active;
  ba.Esrc = w.E[cur];
  ba.Ssrc = w.S[cur];
  ba.Edst = w.E[cur ^ 1];
  ba.Sdst = w.S[cur ^ 1];
  ba.alive = w.alive;
  ba.wind = w.wind;
  ba.zero_count = zero ? &w.count[cur ^ 1] : nullptr;
  ba.m_max = rule.m_max;
  ba.u = rule.u;
  ba.seeds = rule.seeds;
  {
    ProfScope ps("k_band", stream);
    const dim3 g((unsigned)std::min<int64_t>(bound * ntiles, cu_count())), blk(BAND_NW * 64);
    const size_t lds = band_lds(BAND_NW);
    switch (rule.mode()) {
      case BAND_RULE: hipLaunchKernelGGL((k_band_grid<BAND_NW, BAND_RULE>), g, blk, lds, stream, ba, count, ntiles); break;
      case BAND_OPEN: hipLaunchKernelGGL((k_band_grid<BAND_NW, BAND_OPEN>), g, blk, lds, stream, ba, count, ntiles); break;
      default: hipLaunchKernelGGL((k_band_grid<BAND_NW, BAND_PLAIN>), g, blk, lds, stream, ba, count, ntiles);
    }
  }
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((bound + 255) / 256)), dim3(256), 0, stream, k, T_max, cur ^ 1, active,
                     (int)bound, count, w.t_done, w.alive, d_T_dec, w.status, w.active[cur ^ 1], &w.count[cur ^ 1]);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

// First pass of a batch: groups of samples (device lists) with their own
// depth.  Every later pass runs all survivors at the schedule's k_next.
struct FirstPass {
  int nb = 0;
  const int32_t *list[8];
  int count[8];            // group sizes known to the host, or upper bounds when dcount is set
  const int *dcount[8] = {};  // group sizes in device memory (the pass is then sized on the device)
  int k[8];
};

// One batch on the band path: workspace, stream, outputs and first pass.
struct BandRun {
  int L = 0;
  int64_t n = 0;
  int T_max = 0;
  BandWorkspace w;
  FirstPass fp;
  int32_t *T_dec = nullptr;
  uint8_t *flags = nullptr;
  uint32_t *syn = nullptr;
  hipStream_t stream = nullptr;
  Rule rule;
  int cur = 1;
  bool done = false;
  bool device_only = false;  // later passes on the device whatever the setting (no host memory, no wait)
  int64_t first_bound = 0;   // survivors of a first kernel outside fp (the bit-sliced one): an upper bound
};

// Pinned host words for the survivor counts, one block per host thread,
// allocated on first use and kept for the life of the process.
int *pinned_counts(int need) {
  thread_local int *buf = nullptr;
  thread_local int cap = 0;
  if (need > cap) {
    int *p = nullptr;
    const int c = std::max(need, 16);
    if (hipHostMalloc((void **)&p, c * sizeof(int), hipHostMallocDefault) != hipSuccess) return nullptr;
    buf = p;  // an older, smaller block stays allocated (a few bytes)
    cap = c;
  }
  return buf;
}

// Later passes of a batch on the device, with no host wait: DEVICE_GRID_PASSES
// passes over all survivors at once (k_band_grid, tile-parallel, the
// survivor count read on the device), then one launch of k_band_tail for the
// samples still left (one workgroup per sample), then the export.  Full-size
// regions and the schedule's k_next steps per pass throughout.
constexpr int DEVICE_GRID_PASSES = 3;
int band_tail(BandRun &r, int64_t first_count, int grid_passes = DEVICE_GRID_PASSES) {
  const int k = min(schedule_for(r.L).k_next, r.T_max > 0 ? r.T_max : 1);
  BandArgs ba;
  const int nty = tile_geometry(r.L, k, BAND_RY, ba);
  const int ntiles = ba.ntx * nty;
  ba.T_max = r.T_max;
  ba.t_done = r.w.t_done;
  ba.alive = r.w.alive;
  ba.wind = r.w.wind;
  ba.m_max = r.rule.m_max;
  ba.u = r.rule.u;
  ba.seeds = r.rule.seeds;
  int cur = 1;  // the first passes wrote buffer 1 and listed their survivors in active[1]
  for (int pass = 0; pass < grid_passes && first_count > 0; ++pass) {
    ba.active = r.w.active[cur];
    ba.Esrc = r.w.E[cur];
    ba.Ssrc = r.w.S[cur];
    ba.Edst = r.w.E[cur ^ 1];
    ba.Sdst = r.w.S[cur ^ 1];
    ba.zero_count = &r.w.count[cur ^ 1];
    const int64_t grid = std::min<int64_t>(first_count * ntiles, cu_count());
    {
      ProfScope ps("k_band_grid", r.stream);
      const dim3 g((unsigned)grid), blk(BAND_NW * 64);
      const size_t lds = band_lds(BAND_NW);
      const int *cnt = &r.w.count[cur];
      switch (r.rule.mode()) {
        case BAND_RULE:
          hipLaunchKernelGGL((k_band_grid<BAND_NW, BAND_RULE>), g, blk, lds, r.stream, ba, cnt, ntiles);
          break;
        case BAND_OPEN:
          hipLaunchKernelGGL((k_band_grid<BAND_NW, BAND_OPEN>), g, blk, lds, r.stream, ba, cnt, ntiles);
          break;
        default: hipLaunchKernelGGL((k_band_grid<BAND_NW, BAND_PLAIN>), g, blk, lds, r.stream, ba, cnt, ntiles);
      }
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((first_count + 255) / 256)), dim3(256), 0, r.stream, k, r.T_max,
                       cur ^ 1, r.w.active[cur], (int)first_count, (const int *)&r.w.count[cur], r.w.t_done,
                       r.w.alive, r.T_dec, r.w.status, r.w.active[cur ^ 1], &r.w.count[cur ^ 1]);
    HIP_TRY(hipGetLastError());
    cur ^= 1;
  }
  TailArgs ta;
  ta.a = ba;
  ta.a.active = nullptr;
  ta.a.zero_count = nullptr;
  ta.ntiles = ntiles;
  ta.cur = cur;
  for (int b = 0; b < 2; ++b) {
    ta.E[b] = r.w.E[b];
    ta.S[b] = r.w.S[b];
  }
  ta.list = r.w.active[cur];
  ta.count = &r.w.count[cur];
  ta.head = &r.w.count[2];
  ta.t_done = r.w.t_done;
  ta.T_dec = r.T_dec;
  ta.status = r.w.status;
  const int64_t grid = std::min<int64_t>(first_count, cu_count());
  if (grid > 0) {
    ProfScope ps("k_band_tail", r.stream);
    const dim3 g((unsigned)grid), blk(BAND_NW * 64);
    const size_t lds = band_lds(BAND_NW);
    switch (r.rule.mode()) {
      case BAND_RULE: hipLaunchKernelGGL((k_band_tail<BAND_NW, BAND_RULE>), g, blk, lds, r.stream, ta); break;
      case BAND_OPEN: hipLaunchKernelGGL((k_band_tail<BAND_NW, BAND_OPEN>), g, blk, lds, r.stream, ta); break;
      default: hipLaunchKernelGGL((k_band_tail<BAND_NW, BAND_PLAIN>), g, blk, lds, r.stream, ta);
    }
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_band_export, dim3((unsigned)r.n), dim3(256), 0, r.stream, r.L, r.n, r.w.status, r.w.wind,
                     r.w.S[0], r.w.S[1], r.flags, r.syn);
  HIP_TRY(hipGetLastError());
  r.done = true;
  return MPD_OK;
}

// Whether the later passes of a batch run on the device (band_tail) or from
// the host (a survivor-count readback before every pass).  A stream being
// captured into a graph always takes the device: a graph holds no host waits.
bool device_driven(const BandRun &r, int64_t first_count) {
  if (r.device_only) return true;
  const int mode = schedule_for(r.L).driver;
  if (mode == MPD_BAND_DRIVER_DEVICE) return true;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(r.stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return true;
  if (mode == MPD_BAND_DRIVER_HOST) return false;
  (void)first_count;
  return false;
}

// Runs the passes of several band-path batches: the first passes of every
// batch, then, for the batches driven from the host, rounds of one
// survivor-count readback per batch (one host wait per round) and one pass
// for each batch with survivors; batches driven on the device finish with
// one launch.  Batches on different streams overlap on the device.
int band_passes(BandRun *runs, int nr) {
  for (int i = 0; i < nr; ++i) {
    BandRun &r = runs[i];
    bool zero = true;
    for (int b = 0; b < r.fp.nb; ++b) {
      if (r.fp.count[b] == 0) continue;
      const int kb = min(r.fp.k[b], r.T_max > 0 ? r.T_max : 1);
      const int rc = r.fp.dcount[b] != nullptr
                         ? band_pass_dev(r.L, kb, r.T_max, r.w, r.fp.list[b], r.fp.dcount[b], r.fp.count[b], 0, zero,
                                         r.T_dec, r.rule, r.stream)
                         : band_pass(r.L, min(r.fp.k[b], r.T_max), r.T_max, r.w, r.fp.list[b], r.fp.count[b], 0, zero,
                                     r.T_dec, r.rule, r.stream);
      if (rc != MPD_OK) return rc;
      zero = false;
    }
    r.cur = 1;
    r.done = false;
    int64_t first = r.first_bound;
    for (int b = 0; b < r.fp.nb; ++b) first += r.fp.count[b];
    if (device_driven(r, first)) {
      // after the bit-sliced kernel (ten steps) the few survivors go straight
      // to the persistent tail kernel
      const int rc = band_tail(r, first, r.first_bound > 0 ? 0 : DEVICE_GRID_PASSES);
      if (rc != MPD_OK) return rc;
    }
  }
  bool pending = false;
  for (int i = 0; i < nr; ++i) pending = pending || !runs[i].done;
  if (!pending) return MPD_OK;
  int *hc = pinned_counts(nr);
  if (hc == nullptr) return fail_with(MPD_ERR_HIP, "could not allocate pinned host memory for the pass counters");
  for (;;) {
    bool any = false;
    for (int i = 0; i < nr; ++i)
      if (!runs[i].done)
        HIP_TRY(hipMemcpyAsync(&hc[i], &runs[i].w.count[runs[i].cur], sizeof(int), hipMemcpyDeviceToHost,
                               runs[i].stream));
    for (int i = 0; i < nr; ++i)
      if (!runs[i].done) HIP_TRY(hipStreamSynchronize(runs[i].stream));
    for (int i = 0; i < nr; ++i) {
      BandRun &r = runs[i];
      if (r.done) continue;
      if (hc[i] == 0) {
        hipLaunchKernelGGL(k_band_export, dim3((unsigned)r.n), dim3(256), 0, r.stream, r.L, r.n, r.w.status, r.w.wind,
                           r.w.S[0], r.w.S[1], r.flags, r.syn);
        HIP_TRY(hipGetLastError());
        r.done = true;
        continue;
      }
      const int rc = band_pass(r.L, later_pass_k(r.L, hc[i]), r.T_max, r.w, r.w.active[r.cur], hc[i], r.cur, true,
                               r.T_dec, r.rule, r.stream);
      if (rc != MPD_OK) return rc;
      r.cur ^= 1;
      any = true;
    }
    if (!any) break;
  }
  return MPD_OK;
}

// Noise and the first k steps of a plain L = 256 batch in the bit-sliced
// kernel (bits.h), then the usual bookkeeping: T_dec of the samples it
// finished, the survivors' state in buffer 1 and their list in active[1].
// With `order` the workgroups take the samples in that order; with
// `drawn` the noise kernel has already drawn the syndrome into buffer 0 (and
// initialised the bookkeeping), and the kernel reads it instead of drawing.
int bits_start(int L, uint64_t thr, const double *d_p, const uint64_t *d_seeds, int64_t n, int T_max, int k,
               const BandWorkspace &w, int32_t *d_T_dec, hipStream_t stream, const int32_t *order = nullptr,
               bool drawn = false) {
  if (!drawn) {
    hipLaunchKernelGGL(k_tile_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, w.alive, w.wind,
                       w.status, w.t_done, w.active[0], &w.count[2]);
    HIP_TRY(hipGetLastError());
  }
  BitsArgs a = {};
  a.order = order;
  a.S_in = drawn ? w.S[0] : nullptr;
  a.seeds = d_seeds;
  a.thr = thr;
  a.p_arr = d_p;
  a.k = k;
  a.E = w.E[1];
  a.S = w.S[1];
  a.alive = w.alive;
  a.wind = w.wind;
  a.zero_count = &w.count[1];
  {
    ProfScope ps("k_bits", stream);
    if (drawn)
      hipLaunchKernelGGL((k_bits<true, 4>), dim3((unsigned)n), dim3(256), 0, stream, a);
    else
      hipLaunchKernelGGL((k_bits<false, 4>), dim3((unsigned)n), dim3(256), 0, stream, a);
  }
  HIP_TRY(hipGetLastError());
  (void)L;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, k, T_max, 1, w.active[0],
                     (int)n, (const int *)nullptr, w.t_done, w.alive, d_T_dec, w.status, w.active[1], &w.count[1]);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

// The tiled bit-sliced first pass (L > 256) of k steps: the halo they need
// (4k), and tiles per side so that every own part (groups of four rows or
// columns) has at most 256 - 8k sites.
struct TilePlan {
  int k, halo, nt;
};
TilePlan tile_plan(int L, int k) {
  TilePlan t;
  t.k = k;
  t.halo = 4 * k;
  const int own_quads = (256 - 2 * t.halo) / 4;
  t.nt = (L / 4 + own_quads - 1) / own_quads;
  return t;
}

__global__ void k_zero_u2(uint2 *p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_uint2(0u, 0u);
}

// Noise already drawn into buffer 0 (band_start): the first k steps of every
// sample in the tiled bit-sliced kernel, leaving the state in buffer 1 as a
// band first pass would, then T_dec of the finished samples and the list of
// the others in active[1].  With `order` the grid rows take the samples in
// that order.
int bits_tile_start(int L, int64_t n, int T_max, int k, const BandWorkspace &w, int32_t *d_T_dec,
                    hipStream_t stream, const int32_t *order = nullptr) {
  const TilePlan tp = tile_plan(L, k);
  BitsTileArgs a;
  a.L = L;
  a.k = k;
  a.halo = tp.halo;
  a.nt = tp.nt;
  a.order = order;
  a.S_in = w.S[0];
  a.E = w.E[1];
  a.S = w.S[1];
  a.alive = w.alive;
  a.wind = w.wind;
  a.zero_count = &w.count[1];
  // the tiles OR their own rows into the syndrome masks
  const int64_t words = n * (int64_t)(L / TILE_H) * (L / 2);
  hipLaunchKernelGGL(k_zero_u2, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 8192)), dim3(256), 0, stream,
                     w.S[1], words);
  HIP_TRY(hipGetLastError());
  {
    ProfScope ps("k_bits_tile", stream);
    hipLaunchKernelGGL(k_bits_tile, dim3((unsigned)(tp.nt * tp.nt), (unsigned)n), dim3(256), 0, stream, a);
  }
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, k, T_max, 1, w.active[0],
                     (int)n, (const int *)nullptr, w.t_done, w.alive, d_T_dec, w.status, w.active[1], &w.count[1]);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

// Noise (or explicit errors) and first-pass setup of a plain (single-group) band batch.
int band_setup(BandRun &r, int L, uint64_t thr, const double *d_p, const uint64_t *d_seeds, int64_t n, int T_max,
               int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_syn, void *ws, hipStream_t stream,
               const uint32_t *d_links = nullptr) {
  r.L = L;
  r.n = n;
  r.T_max = T_max;
  r.w = band_layout(L, n, ws);
  r.T_dec = d_T_dec;
  r.flags = d_flags;
  r.syn = d_syn;
  r.stream = stream;
  const int kb = schedule_for(L).k_bits;
  if (L == BITS_L && kb > 0 && d_links == nullptr && r.rule.mode() == BAND_PLAIN) {
    // noise and the first min(k_bits, T_max) steps in the bit-sliced kernel,
    // which leaves the survivors in buffer 1 as a band first pass would
    r.fp.nb = 0;
    r.first_bound = n;
    return bits_start(L, thr, d_p, d_seeds, n, T_max, std::min(kb, T_max), r.w, d_T_dec, stream);
  }
  if (L > BITS_L && kb > 0 && T_max > 0 && d_links == nullptr && r.rule.mode() == BAND_PLAIN) {
    // noise, then the first min(k_bits, T_max) steps in the tiled bit-sliced kernel
    const int rc = band_start(L, thr, d_p, d_seeds, n, r.w, nullptr, stream);
    if (rc != MPD_OK) return rc;
    r.fp.nb = 0;
    r.first_bound = n;
    return bits_tile_start(L, n, T_max, std::min(std::min(kb, T_max), BITS_TILE_MAX_STEPS), r.w, d_T_dec, stream);
  }
  r.fp.nb = 1;
  r.fp.list[0] = r.w.active[0];
  r.fp.count[0] = (int)n;
  r.fp.k[0] = schedule_for(L).k_first;
  return band_start(L, thr, d_p, d_seeds, n, r.w, nullptr, stream, r.rule.open ? 1 : 0, d_links);
}

int decode_band(int L, uint64_t thr, const double *d_p, const uint64_t *d_seeds, int64_t n, int T_max,
                int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_syn, void *ws, const Rule &rule, hipStream_t stream) {
  BandRun r;
  r.rule = rule;
  const int rc = band_setup(r, L, thr, d_p, d_seeds, n, T_max, d_T_dec, d_flags, d_syn, ws, stream);
  if (rc != MPD_OK) return rc;
  return band_passes(&r, 1);
}

// Exactly t_exact decoder steps from step t_start for every sample on the
// band path (no early exit, no compaction): passes of up to k_first steps
// over all samples, the state alternating between the two buffers.  The
// initial state is in buffer 0; returns the buffer that holds the final one.
int band_run_exact(int L, int64_t n, int t_start, int t_exact, const BandWorkspace &w, const Rule &rule,
                   hipStream_t stream, int *final_buf) {
  const int t_end = t_start + t_exact;
  const int kf = schedule_for(L).k_first;
  int cur = 0;
  for (int t = t_start; t < t_end;) {
    const int k = std::min(kf, t_end - t);
    BandArgs ba;
    const int nty = tile_geometry(L, k, BAND_RY, ba);
    ba.T_max = t_end;
    ba.t_done = w.t_done;
    ba.active = w.active[0];
    ba.Esrc = w.E[cur];
    ba.Ssrc = w.S[cur];
    ba.Edst = w.E[cur ^ 1];
    ba.Sdst = w.S[cur ^ 1];
    ba.alive = w.alive;
    ba.wind = w.wind;
    ba.zero_count = nullptr;
    ba.m_max = rule.m_max;
    ba.u = rule.u;
    ba.seeds = rule.seeds;
    {
      ProfScope ps("k_band", stream);
      const dim3 grid((unsigned)(ba.ntx * nty), (unsigned)n), blk(BAND_NW * 64);
      const size_t lds = band_lds(BAND_NW);
      if (rule.on())
        hipLaunchKernelGGL((k_band<BAND_NW, BAND_RULE>), grid, blk, lds, stream, ba);
      else
        hipLaunchKernelGGL((k_band<BAND_NW, BAND_PLAIN>), grid, blk, lds, stream, ba);
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_band_advance, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, k, t_end,
                       w.t_done, w.alive);
    HIP_TRY(hipGetLastError());
    cur ^= 1;
    t += k;
  }
  *final_buf = cur;
  return MPD_OK;
}

// Library-owned side streams (default priority, non-blocking) with
// fork/join events, created on first use and kept for the process.
constexpr int BAND_STREAMS = 4;
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipStream_t band[BAND_STREAMS] = {};   // band-path classes of a mixed batch
  hipEvent_t band_join[BAND_STREAMS] = {};
};
// Per host thread and device, so that concurrent calls from several threads
// never share streams or fork/join events.
thread_local std::map<int, SideStream> t_side;

SideStream *side_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  auto it = t_side.find(dev);
  if (it != t_side.end()) return &it->second;
  SideStream s;
  if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&s.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&s.join, hipEventDisableTiming) != hipSuccess) return nullptr;
  for (int i = 0; i < BAND_STREAMS; ++i) {
    if (hipStreamCreateWithFlags(&s.band[i], hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&s.band_join[i], hipEventDisableTiming) != hipSuccess) return nullptr;
  }
  return &(t_side[dev] = s);
}

int check_common(int L, int64_t n, int T_max, const void *T_dec, const void *flags) {
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "n=%lld out of range", (long long)n);
  if (T_max < 0 || T_max > MPD_T_MAX_LIMIT)
    return fail_with(MPD_ERR_TMAX, "T_max=%d outside [0, %d]", T_max, MPD_T_MAX_LIMIT);
  if (n > 0 && (T_dec == nullptr || flags == nullptr))
    return fail_with(MPD_ERR_PTR, "T_dec and flags must not be NULL");
  if (((uintptr_t)T_dec & 3u) != 0) return fail_with(MPD_ERR_PTR, "T_dec must be 4-byte aligned");
  (void)L;
  return MPD_OK;
}

// ---------------------------------------------------------------------------
// Learned scheduling: predicted decode time -> first-pass depth per group
// ---------------------------------------------------------------------------

constexpr int MAX_BINS = 8;
struct BinEdges {
  float v[MAX_BINS - 1];
};

// Sample i goes to bin b with edges[b-1] <= pred[i] < edges[b] (bin 0 below
// the first edge, NaN included); lists [nb][n], counts [nb] zero on entry.
__global__ void k_bin(const float *pred, int64_t n, int nb, BinEdges e, int32_t *lists, int *counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  int b = -1;
  if (in) {
    const float v = pred[i];
    b = 0;
    while (b < nb - 1 && v >= e.v[b]) ++b;
  }
  // one atomic per wave and bin: the wave's members of bin c take consecutive slots
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < nb; ++c) {
    const uint64_t m = __ballot(b == c);
    if (m == 0) continue;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[c], __popcll(m));
    base = __shfl(base, leader);
    if (b == c) lists[(int64_t)c * n + base + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
  }
}

// The groups' lists one after another, from the group with the longest
// predicted decoding time to the shortest: the order in which the bit-sliced
// kernel takes the samples (longest first, so they do not form the tail).
__global__ void k_order(const int32_t *lists, const int *counts, int nb, int64_t n, int32_t *order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t off = 0;
  for (int b = nb - 1; b >= 0; --b) {
    const int64_t c = counts[b];
    if (i < off + c) {
      order[i] = lists[(int64_t)b * n + (i - off)];
      return;
    }
    off += c;
  }
}

__global__ void k_zero_i32(int *p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

// Workspace of a learned-schedule decode: the band workspace followed by the
// block counts, predictions, bin lists and the predictor's own workspace.
struct LearnedLayout {
  BandWorkspace band;
  uint8_t *counts;
  float *pred;
  int32_t *lists;
  int *bin_count;
  int32_t *order;
  void *cnn_ws;
  size_t bytes;
};
LearnedLayout learned_layout(int L, int64_t n, void *base) {
  LearnedLayout l;
  l.band = band_layout(L, n, base);
  size_t off = l.band.bytes;
  auto take = [&](size_t bytes) {
    void *p = base ? (void *)((char *)base + off) : nullptr;
    off += align256(bytes);
    return p;
  };
  const int M = L / 8;
  l.counts = (uint8_t *)take((size_t)n * M * M);
  l.pred = (float *)take((size_t)n * 4);
  l.lists = (int32_t *)take((size_t)MAX_BINS * n * 4);
  l.bin_count = (int *)take(MAX_BINS * sizeof(int));
  l.order = (int32_t *)take((size_t)n * 4);
  l.cnn_ws = take(cnn_forward_ws(M, n));
  l.bytes = off;
  return l;
}

// Library-held scratch of the allocation-free decode (mpd_decode_batch_static):
// the band path's state and bookkeeping for up to MPD_STATIC_SCRATCH_BYTES.
// Each device the library runs on holds its own copy until the process
// ends.  Host code never passes `scratch` itself (on the host it only names
// the symbol): it looks the device address up once per device and passes
// that pointer to the kernels.
static __device__ __align__(256) unsigned char scratch[MPD_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on the current device, looked up on
// the first call for that device (with it current), then reused.  The
// compute-unit count is cached at the same time, so that later calls touch
// no allocating container.
int static_scratch(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail_with(MPD_ERR_HIP, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr || ((uintptr_t)p & 255u)) return fail_with(MPD_ERR_HIP, "scratch symbol has no usable address");
    (void)cu_count();
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MPD_OK;
}

}  // namespace mpd

using namespace mpd;

extern "C" {

const char *mpd_version(void) { return "mpd 0.1 gfx950"; }

const char *mpd_last_error(void) { return g_last_error.c_str(); }

size_t mpd_workspace_bytes(int L, int64_t n) {
  if (n <= 0) return 0;
  if (resident_ok(L)) return 0;
  if (tiled_ok(L)) return band_layout(L, n, nullptr).bytes;
  return 0;
}

// Range of the limited-memory parameters.
static int check_rule(int m_max, int u) {
  if (m_max < 0 || u < 0) return fail_with(MPD_ERR_RULE, "m_max=%d, u=%d: both must be >= 0", m_max, u);
  return MPD_OK;
}

static int decode_seeded(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, const Rule &rule,
                  int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_final_syndrome, void *d_workspace,
                  size_t ws_bytes, void *stream) {
  if (!(p >= 0.0 && p <= 1.0)) return fail_with(MPD_ERR_P, "p must lie in [0, 1]");
  int rc = check_common(L, n, T_max, d_T_dec, d_flags);
  if (rc) return rc;
  if (!resident_ok(L) && !tiled_ok(L))
    return fail_with(MPD_ERR_L, "L=%d unsupported (3..128 with a strip height, or a multiple of 16 in [256, 16384])", L);
  if (n == 0) return MPD_OK;
  if (d_seeds == nullptr || ((uintptr_t)d_seeds & 7u)) return fail_with(MPD_ERR_PTR, "seeds NULL or misaligned");
  if (d_final_syndrome != nullptr && ((uintptr_t)d_final_syndrome & 3u))
    return fail_with(MPD_ERR_PTR, "final_syndrome misaligned");
  const uint64_t thr = threshold_of(p);
  hipStream_t st = (hipStream_t)stream;
  if (resident_ok(L)) {
    if (!rule.on())
      return launch_small(L, n, d_seeds, thr, nullptr, T_max, d_T_dec, d_flags, d_final_syndrome, st);
    ResidentArgs a = {};
    a.L = L;
    a.n = n;
    a.seeds = d_seeds;
    a.thr = thr;
    a.p_arr = nullptr;
    a.links = nullptr;
    a.T_max = T_max;
    a.t_exact = -1;
    a.T_dec = d_T_dec;
    a.flags = d_flags;
    a.syn = d_final_syndrome;
    a.m_max = rule.m_max;
    a.u = rule.u;
    return launch_resident(a, st);
  }
  if (n > BAND_MAX_N) return fail_with(MPD_ERR_N, "n=%lld: at most %d samples per band-path call", (long long)n, BAND_MAX_N);
  const size_t need = mpd_workspace_bytes(L, n);
  if (ws_bytes < need || d_workspace == nullptr)
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
  if ((uintptr_t)d_workspace & 255u) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  return decode_band(L, thr, nullptr, d_seeds, n, T_max, d_T_dec, d_flags, d_final_syndrome, d_workspace, rule, st);
}

int mpd_decode_batch(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int32_t *d_T_dec,
                     uint8_t *d_flags, uint32_t *d_final_syndrome, void *d_workspace, size_t ws_bytes,
                     void *stream) {
  g_last_error.clear();
  return decode_seeded(L, p, d_seeds, n, T_max, Rule(), d_T_dec, d_flags, d_final_syndrome, d_workspace, ws_bytes,
                       stream);
}

int mpd_decode_batch_static(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int32_t *d_T_dec,
                            uint8_t *d_flags, uint32_t *d_final_syndrome, void *stream) {
  g_last_error.clear();
  if (!(p >= 0.0 && p <= 1.0)) return fail_with(MPD_ERR_P, "p must lie in [0, 1]");
  int rc = check_common(L, n, T_max, d_T_dec, d_flags);
  if (rc) return rc;
  if (!resident_ok(L) && !tiled_ok(L))
    return fail_with(MPD_ERR_L, "L=%d unsupported (3..128 with a strip height, or a multiple of 16 in [256, 16384])", L);
  if (n == 0) return MPD_OK;
  if (d_seeds == nullptr || ((uintptr_t)d_seeds & 7u)) return fail_with(MPD_ERR_PTR, "seeds NULL or misaligned");
  if (d_final_syndrome != nullptr && ((uintptr_t)d_final_syndrome & 3u))
    return fail_with(MPD_ERR_PTR, "final_syndrome misaligned");
  hipStream_t st = (hipStream_t)stream;
  if (resident_ok(L))  // decodes on chip: no scratch at all
    return launch_small(L, n, d_seeds, threshold_of(p), nullptr, T_max, d_T_dec, d_flags, d_final_syndrome, st);
  if (n > BAND_MAX_N) return fail_with(MPD_ERR_N, "n=%lld: at most %d samples per band-path call", (long long)n, BAND_MAX_N);
  const size_t need = mpd_workspace_bytes(L, n);
  if (need > (size_t)MPD_STATIC_SCRATCH_BYTES)
    return fail_with(MPD_ERR_WORKSPACE,
                     "L=%d, n=%lld needs %zu bytes of scratch; the library holds %zu (use mpd_decode_batch with a "
                     "workspace)", L, (long long)n, need, (size_t)MPD_STATIC_SCRATCH_BYTES);
  void *ws = nullptr;
  rc = static_scratch(&ws);
  if (rc != MPD_OK) return rc;
  BandRun r;
  r.device_only = true;
  rc = band_setup(r, L, threshold_of(p), nullptr, d_seeds, n, T_max, d_T_dec, d_flags, d_final_syndrome, ws, st);
  if (rc != MPD_OK) return rc;
  return band_passes(&r, 1);
}

int mpd_decode_rule(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int m_max, int u,
                    int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_final_syndrome, void *d_workspace,
                    size_t ws_bytes, void *stream) {
  g_last_error.clear();
  const int rc = check_rule(m_max, u);
  if (rc) return rc;
  Rule rule;
  rule.m_max = m_max;
  rule.u = u;
  rule.seeds = d_seeds;
  return decode_seeded(L, p, d_seeds, n, T_max, rule, d_T_dec, d_flags, d_final_syndrome, d_workspace, ws_bytes,
                       stream);
}

int mpd_syndrome_counts(int L, double p, const double *d_p, const uint64_t *d_seeds, int64_t n, uint8_t *d_counts,
                        void *stream) {
  g_last_error.clear();
  if (L < 16 || L > 16384 || L % 16) return fail_with(MPD_ERR_L, "L=%d: need a multiple of 16 in [16, 16384]", L);
  if (d_p == nullptr && !(p >= 0.0 && p <= 1.0)) return fail_with(MPD_ERR_P, "p must lie in [0, 1]");
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "n=%lld out of range", (long long)n);
  if (n == 0) return MPD_OK;
  if (d_seeds == nullptr || ((uintptr_t)d_seeds & 7u) || d_counts == nullptr || ((uintptr_t)d_p & 7u))
    return fail_with(MPD_ERR_PTR, "seeds/counts NULL or misaligned");
  const NoiseShape g = noise_shape(L);
  hipLaunchKernelGGL(k_band_noise<false>, dim3((unsigned)(n * g.groups)), dim3(g.CP * g.S), g.lds,
                     (hipStream_t)stream, L, g.CP, g.S, d_seeds, threshold_of(d_p ? 0.0 : p), d_p, (uint2 *)nullptr,
                     (uint32_t *)nullptr, d_counts);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

size_t mpd_learned_workspace_bytes(int L, int64_t n) {
  if (n <= 0 || !tiled_ok(L)) return 0;
  return learned_layout(L, n, nullptr).bytes;
}

int mpd_decode_learned(int L, double p, const double *d_p, const uint64_t *d_seeds, int64_t n, int T_max,
                       const float *d_params, int n_bins, const float *h_edges, const int *h_depth, int32_t *d_T_dec,
                       uint8_t *d_flags, uint32_t *d_final_syndrome, float *d_pred, void *d_workspace,
                       size_t ws_bytes, void *stream) {
  g_last_error.clear();
  if (d_p == nullptr && !(p >= 0.0 && p <= 1.0)) return fail_with(MPD_ERR_P, "p must lie in [0, 1]");
  int rc = check_common(L, n, T_max, d_T_dec, d_flags);
  if (rc) return rc;
  if (!tiled_ok(L)) return fail_with(MPD_ERR_L, "L=%d: learned scheduling needs a multiple of 16 in [256, 16384]", L);
  if (n > BAND_MAX_N) return fail_with(MPD_ERR_N, "n=%lld: at most %d samples per band-path call", (long long)n, BAND_MAX_N);
  if (n_bins < 1 || n_bins > MAX_BINS) return fail_with(MPD_ERR_N, "n_bins=%d outside [1, %d]", n_bins, MAX_BINS);
  if (h_depth == nullptr || (n_bins > 1 && h_edges == nullptr)) return fail_with(MPD_ERR_PTR, "NULL policy");
  BinEdges e;
  for (int b = 0; b < n_bins; ++b) {
    if (h_depth[b] < 1 || 4 * h_depth[b] >= BAND_RX / 2)
      return fail_with(MPD_ERR_TMAX, "bin depth %d outside [1, 15]", h_depth[b]);
    if (b + 1 < n_bins) {
      e.v[b] = h_edges[b];
      if (!(e.v[b] == e.v[b]) || (b > 0 && e.v[b] < e.v[b - 1]))
        return fail_with(MPD_ERR_P, "bin edges must be ascending numbers");
    }
  }
  if (n == 0) return MPD_OK;
  if (d_seeds == nullptr || ((uintptr_t)d_seeds & 7u) || d_params == nullptr || ((uintptr_t)d_params & 3u) ||
      ((uintptr_t)d_pred & 3u) || ((uintptr_t)d_final_syndrome & 3u) || ((uintptr_t)d_p & 7u))
    return fail_with(MPD_ERR_PTR, "seeds/params/pred/syndrome/p NULL or misaligned");
  const LearnedLayout l = learned_layout(L, n, d_workspace);
  if (d_workspace == nullptr || ws_bytes < l.bytes)
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, l.bytes);
  if ((uintptr_t)d_workspace & 255u) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  if (n_bins == 1 && d_pred == nullptr) {
    // One group and no predictions asked for: nothing would read the
    // network's output, so this is the plain decode (FIFO) at the group's
    // first-pass depth, without inference.
    BandRun r;
    rc = band_setup(r, L, threshold_of(d_p ? 0.0 : p), d_p, d_seeds, n, T_max, d_T_dec, d_flags, d_final_syndrome,
                    d_workspace, st);
    if (rc != MPD_OK) return rc;
    r.fp.k[0] = h_depth[0];
    return band_passes(&r, 1);
  }
  rc = band_start(L, threshold_of(d_p ? 0.0 : p), d_p, d_seeds, n, l.band, l.counts, st);
  if (rc != MPD_OK) return rc;
  rc = cnn_forward_run(l.counts, L / 8, n, d_params, l.pred, nullptr, nullptr, nullptr, l.cnn_ws, st);
  if (rc != MPD_OK) return rc;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, l.bin_count, MAX_BINS);
  hipLaunchKernelGGL(k_bin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, l.pred, n, n_bins, e, l.lists,
                     l.bin_count);
  HIP_TRY(hipGetLastError());
  if (d_pred != nullptr) HIP_TRY(hipMemcpyAsync(d_pred, l.pred, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  const int kb = schedule_for(L).k_bits;
  if (kb > 0 && (L == BITS_L || T_max > 0)) {
    // the bit-sliced kernel stops each sample when it has no anyon, so the
    // groups set the order in which it takes them (longest predicted first),
    // not a depth; it reads the syndrome the noise kernel drew.  (The tiled
    // kernel for L > 256 runs the same number of steps on every sample: the
    // order only sets which samples its grid takes first.)
    hipLaunchKernelGGL(k_order, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, l.lists, l.bin_count, n_bins,
                       n, l.order);
    HIP_TRY(hipGetLastError());
    BandRun r;
    r.L = L;
    r.n = n;
    r.T_max = T_max;
    r.w = l.band;
    r.T_dec = d_T_dec;
    r.flags = d_flags;
    r.syn = d_final_syndrome;
    r.stream = st;
    r.fp.nb = 0;
    r.first_bound = n;
    if (L == BITS_L)
      rc = bits_start(L, 0, nullptr, d_seeds, n, T_max, std::min(kb, T_max), r.w, d_T_dec, st, l.order, true);
    else
      rc = bits_tile_start(L, n, T_max, std::min(std::min(kb, T_max), BITS_TILE_MAX_STEPS), r.w, d_T_dec, st,
                           l.order);
    if (rc != MPD_OK) return rc;
    return band_passes(&r, 1);
  }
  BandRun r;
  r.L = L;
  r.n = n;
  r.T_max = T_max;
  r.w = l.band;
  r.T_dec = d_T_dec;
  r.flags = d_flags;
  r.syn = d_final_syndrome;
  r.stream = st;
  r.fp.nb = n_bins;
  // the group sizes stay on the device: each group's first pass is sized
  // there (no host wait before the first passes)
  for (int b = 0; b < n_bins; ++b) {
    r.fp.count[b] = (int)n;
    r.fp.dcount[b] = l.bin_count + b;
    r.fp.list[b] = l.lists + (int64_t)b * n;
    r.fp.k[b] = h_depth[b];
  }
  return band_passes(&r, 1);
}

int mpd_profile(int enable) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (enable) {
    for (auto &r : g_prof.recs) {
      g_prof.pool.push_back(r.a);
      g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
  }
  g_prof.on = enable != 0;
  return MPD_OK;
}

int mpd_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
  g_last_error.clear();
  if (kernel == nullptr || total_ms == nullptr || launches == nullptr)
    return fail_with(MPD_ERR_PTR, "profile_read arguments must not be NULL");
  double ms = 0.0;
  int64_t cnt = 0;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto &r : g_prof.recs) {
    if (strcmp(r.name, kernel) != 0) continue;
    HIP_TRY(hipEventSynchronize(r.b));
    float e = 0.f;
    HIP_TRY(hipEventElapsedTime(&e, r.a, r.b));
    ms += e;
    ++cnt;
  }
  *total_ms = ms;
  *launches = cnt;
  return MPD_OK;
}

int mpd_set_band_schedule(int L, int k_first, int k_next) {
  g_last_error.clear();
  // the halo 4k must leave owned columns in a 128-column region
  if (k_first < 1 || k_next < 1 || 4 * k_first >= BAND_RX / 2 || 4 * k_next >= BAND_RX / 2)
    return fail_with(MPD_ERR_TMAX, "steps per pass must be in [1, 15]");
  std::lock_guard<std::mutex> lk(g_sched_mu);
  if (L == 0) {
    g_sched_default.k_first = k_first;
    g_sched_default.k_next = k_next;
    g_sched_by_L.clear();
  } else {
    auto it = g_sched_by_L.find(L);
    BandSchedule b = it == g_sched_by_L.end() ? g_sched_default : it->second;
    b.k_first = k_first;
    b.k_next = k_next;
    g_sched_by_L[L] = b;
  }
  return MPD_OK;
}

int mpd_set_band_driver(int L, int driver) {
  g_last_error.clear();
  if (driver != MPD_BAND_DRIVER_AUTO && driver != MPD_BAND_DRIVER_HOST && driver != MPD_BAND_DRIVER_DEVICE)
    return fail_with(MPD_ERR_N, "driver %d: use MPD_BAND_DRIVER_AUTO, _HOST or _DEVICE", driver);
  std::lock_guard<std::mutex> lk(g_sched_mu);
  if (L == 0) {
    g_sched_default.driver = driver;
    for (auto &kv : g_sched_by_L) kv.second.driver = driver;
  } else {
    auto it = g_sched_by_L.find(L);
    BandSchedule b = it == g_sched_by_L.end() ? g_sched_default : it->second;
    b.driver = driver;
    g_sched_by_L[L] = b;
  }
  return MPD_OK;
}

int mpd_get_band_driver(int L, int *driver) {
  g_last_error.clear();
  if (driver == nullptr) return fail_with(MPD_ERR_PTR, "NULL output");
  *driver = schedule_for(L).driver;
  return MPD_OK;
}

int mpd_get_band_schedule(int L, int *k_first, int *k_next) {
  g_last_error.clear();
  if (k_first == nullptr || k_next == nullptr) return fail_with(MPD_ERR_PTR, "NULL output");
  const BandSchedule b = schedule_for(L);
  *k_first = b.k_first;
  *k_next = b.k_next;
  return MPD_OK;
}

int mpd_set_band_bits(int L, int k_bits) {
  g_last_error.clear();
  if (k_bits < 0 || k_bits > BITS_MAX_STEPS) return fail_with(MPD_ERR_TMAX, "bit-sliced steps must be in [0, %d]", BITS_MAX_STEPS);
  std::lock_guard<std::mutex> lk(g_sched_mu);
  if (L == 0) {
    g_sched_default.k_bits = k_bits;
    for (auto &kv : g_sched_by_L) kv.second.k_bits = k_bits;
  } else {
    auto it = g_sched_by_L.find(L);
    BandSchedule b = it == g_sched_by_L.end() ? g_sched_default : it->second;
    b.k_bits = k_bits;
    g_sched_by_L[L] = b;
  }
  return MPD_OK;
}

int mpd_get_band_bits(int L, int *k_bits) {
  g_last_error.clear();
  if (k_bits == nullptr) return fail_with(MPD_ERR_PTR, "NULL output");
  *k_bits = schedule_for(L).k_bits;
  return MPD_OK;
}

int mpd_autotune_band(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int32_t *d_T_dec,
                      uint8_t *d_flags, void *d_workspace, size_t ws_bytes, void *stream, int *k_first,
                      int *k_next, float *best_ms) {
  g_last_error.clear();
  if (!tiled_ok(L)) return fail_with(MPD_ERR_L, "autotuning applies to the band path (L >= 256)");
  if (k_first == nullptr || k_next == nullptr || best_ms == nullptr) return fail_with(MPD_ERR_PTR, "NULL output");
  if (n <= 0) return fail_with(MPD_ERR_N, "autotuning needs a non-empty probe batch");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const BandSchedule saved = schedule_for(L);
  bool had = false;
  {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    had = g_sched_by_L.count(L) != 0;
  }
  float best = 1e30f;
  BandSchedule pick = saved;
  int rc = MPD_OK;
  // candidates: driver x (steps of the bit-sliced first kernel: 0, 3, 5, 8,
  // 10 at L = 256; of the tiled one, 0, 4, 5, 6, above) x first-pass depth 1..8
  // (only without a bit-sliced kernel: with it the band passes start later)
  // x later depth 1..8
  std::vector<BandSchedule> cand;
  const bool bits_here = L == BITS_L, tiles_here = L > BITS_L;
  for (int drv = MPD_BAND_DRIVER_HOST; drv <= MPD_BAND_DRIVER_DEVICE; ++drv)
    for (int kb : {0, 3, 4, 5, 6, 8, 10}) {
      if (bits_here ? (kb == 4 || kb == 6) : tiles_here ? (kb == 3 || kb > 6) : kb != 0) continue;
      for (int kf = 1; kf <= 8; ++kf) {
        if (kb > 0 && kf != saved.k_first) continue;
        for (int kn = 1; kn <= 8; ++kn) {
          BandSchedule c;
          c.k_first = kf;
          c.k_next = kn;
          c.driver = drv;
          c.k_bits = (bits_here || tiles_here) ? kb : saved.k_bits;
          cand.push_back(c);
        }
      }
    }
  // one probe decode under schedule c, after a warm-up decode under it
  auto time_one = [&](const BandSchedule &c, float &ms) -> int {
    {
      std::lock_guard<std::mutex> lk(g_sched_mu);
      g_sched_by_L[L] = c;
    }
    int r = mpd_decode_batch(L, p, d_seeds, n, T_max, d_T_dec, d_flags, nullptr, d_workspace, ws_bytes, stream);
    if (r) return r;
    if (hipEventRecord(e0, st) != hipSuccess) return fail_with(MPD_ERR_HIP, "event record");
    r = mpd_decode_batch(L, p, d_seeds, n, T_max, d_T_dec, d_flags, nullptr, d_workspace, ws_bytes, stream);
    if (r) return r;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return fail_with(MPD_ERR_HIP, "event timing");
    ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return MPD_OK;
  };
  // Screening: one timed decode per candidate.  The minimum of many single
  // timings of a short probe favours whichever candidate met a quiet moment,
  // so the fastest few are timed again in interleaved rounds and the pick is
  // the lowest median.
  constexpr int FINALISTS = 8, ROUNDS = 5;
  std::vector<float> first(cand.size(), 1e30f);
  for (size_t ci = 0; ci < cand.size() && rc == MPD_OK; ++ci) rc = time_one(cand[ci], first[ci]);
  if (rc == MPD_OK) {
    std::vector<size_t> order(cand.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return first[x] < first[y]; });
    order.resize(std::min<size_t>(order.size(), FINALISTS));
    std::vector<std::vector<float>> again(order.size());
    for (int r = 0; r < ROUNDS && rc == MPD_OK; ++r)
      for (size_t f = 0; f < order.size() && rc == MPD_OK; ++f) {
        float ms = 0.f;
        rc = time_one(cand[order[f]], ms);
        again[f].push_back(ms);
      }
    for (size_t f = 0; f < order.size() && rc == MPD_OK; ++f) {
      std::vector<float> v = again[f];
      std::sort(v.begin(), v.end());
      const float med = v[v.size() / 2];
      if (med < best) {
        best = med;
        pick = cand[order[f]];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    if (rc == MPD_OK) g_sched_by_L[L] = pick;
    else if (had) g_sched_by_L[L] = saved;
    else g_sched_by_L.erase(L);
  }
  if (rc) return rc;
  *k_first = pick.k_first;
  *k_next = pick.k_next;
  *best_ms = best;
  return MPD_OK;
}

size_t mpd_mixed_workspace_bytes(int n_classes, const int32_t *h_L, const int64_t *h_count) {
  size_t need = 0;
  if (n_classes <= 0 || h_L == nullptr || h_count == nullptr) return 0;
  for (int c = 0; c < n_classes; ++c)  // band classes run concurrently, each with its own part
    if (!resident_ok(h_L[c]) && tiled_ok(h_L[c])) need += align256(mpd_workspace_bytes(h_L[c], h_count[c]));
  return need;
}

int mpd_decode_mixed(int n_classes, const int32_t *h_L, const int64_t *h_count, const double *d_p,
                     const uint64_t *d_seeds, int T_max, int32_t *d_T_dec, uint8_t *d_flags,
                     uint32_t *d_final_syndrome, void *d_workspace, size_t ws_bytes, void *stream) {
  g_last_error.clear();
  if (n_classes < 0 || (n_classes > 0 && (h_L == nullptr || h_count == nullptr)))
    return fail_with(MPD_ERR_PTR, "class arrays must not be NULL");
  int64_t n = 0;
  for (int c = 0; c < n_classes; ++c) {
    if (!resident_ok(h_L[c]) && !tiled_ok(h_L[c])) return fail_with(MPD_ERR_L, "class %d: L=%d unsupported", c, h_L[c]);
    if (h_count[c] < 0) return fail_with(MPD_ERR_N, "class %d: negative count", c);
    if (!resident_ok(h_L[c]) && h_count[c] > BAND_MAX_N)
      return fail_with(MPD_ERR_N, "class %d: at most %d samples of a band-path size", c, BAND_MAX_N);
    n += h_count[c];
  }
  int rc = check_common(4, n, T_max, d_T_dec, d_flags);
  if (rc) return rc;
  if (n == 0) return MPD_OK;
  if (d_p == nullptr || d_seeds == nullptr || ((uintptr_t)d_seeds & 7u) || ((uintptr_t)d_p & 7u))
    return fail_with(MPD_ERR_PTR, "p and seeds must be non-NULL and 8-byte aligned");
  const size_t need = mpd_mixed_workspace_bytes(n_classes, h_L, h_count);
  if (need > 0 && (ws_bytes < need || d_workspace == nullptr))
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
  if (need > 0 && ((uintptr_t)d_workspace & 255u)) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  {
    // A batch of one size: no fork onto the side streams, one decode on
    // `stream` (the band workspace then starts at d_workspace).
    int nz = 0, c1 = -1;
    int64_t off1 = 0, syn1 = 0, o = 0, so = 0;
    for (int c = 0; c < n_classes; ++c) {
      if (h_count[c] > 0) {
        ++nz;
        c1 = c;
        off1 = o;
        syn1 = so;
      }
      o += h_count[c];
      so += h_count[c] * (((int64_t)h_L[c] * h_L[c] + 31) / 32);
    }
    if (nz == 1) {
      const int L = h_L[c1];
      const int64_t cnt = h_count[c1];
      uint32_t *syn = d_final_syndrome ? d_final_syndrome + syn1 : nullptr;
      if (!resident_ok(L))
        return decode_band(L, 0, d_p + off1, d_seeds + off1, cnt, T_max, d_T_dec + off1, d_flags + off1, syn,
                           d_workspace, Rule(), st);
      return launch_small(L, cnt, d_seeds + off1, 0, d_p + off1, T_max, d_T_dec + off1, d_flags + off1, syn, st);
    }
  }
  SideStream *side = side_stream();
  if (side == nullptr) return fail_with(MPD_ERR_HIP, "could not create the side stream");
  // fork: resident classes on the side stream
  HIP_TRY(hipEventRecord(side->fork, st));
  HIP_TRY(hipStreamWaitEvent(side->stream, side->fork, 0));
  int64_t off = 0, syn_off = 0;
  for (int c = 0; c < n_classes; ++c) {
    const int L = h_L[c];
    const int64_t cnt = h_count[c];
    if (cnt > 0 && resident_ok(L)) {
      rc = launch_small(L, cnt, d_seeds + off, 0, d_p + off, T_max, d_T_dec + off, d_flags + off,
                        d_final_syndrome ? d_final_syndrome + syn_off : nullptr, side->stream);
      if (rc) return rc;
    }
    off += cnt;
    syn_off += cnt * (((int64_t)L * L + 31) / 32);
  }
  HIP_TRY(hipEventRecord(side->join, side->stream));
  // band classes: each on a stream of the pool with its own workspace part,
  // passes in lockstep
  std::vector<BandRun> runs;
  off = 0;
  syn_off = 0;
  size_t ws_off = 0;
  for (int c = 0; c < n_classes; ++c) {
    const int L = h_L[c];
    const int64_t cnt = h_count[c];
    if (cnt > 0 && !resident_ok(L)) {
      const int si = (int)(runs.size() % BAND_STREAMS);
      HIP_TRY(hipStreamWaitEvent(side->band[si], side->fork, 0));
      runs.emplace_back();
      rc = band_setup(runs.back(), L, 0, d_p + off, d_seeds + off, cnt, T_max, d_T_dec + off, d_flags + off,
                      d_final_syndrome ? d_final_syndrome + syn_off : nullptr, (char *)d_workspace + ws_off,
                      side->band[si]);
      if (rc) return rc;
      ws_off += align256(mpd_workspace_bytes(L, cnt));
    }
    off += cnt;
    syn_off += cnt * (((int64_t)L * L + 31) / 32);
  }
  if (!runs.empty()) {
    rc = band_passes(runs.data(), (int)runs.size());
    if (rc) return rc;
    for (int i = 0; i < std::min((int)runs.size(), BAND_STREAMS); ++i) {
      HIP_TRY(hipEventRecord(side->band_join[i], side->band[i]));
      HIP_TRY(hipStreamWaitEvent(st, side->band_join[i], 0));
    }
  }
  HIP_TRY(hipStreamWaitEvent(st, side->join, 0));
  return MPD_OK;
}

// Open lattices need the zero row in LDS too.
static bool open_ok(int L) { return resident_ok(L) && resident_lds(L, resident_H(L), true) <= 160 * 1024; }

static int decode_links_rule(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n, int T_max,
                      int m_max, int u, int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_final_syndrome,
                      void *stream, int open = 0) {
  int rc = check_common(L, n, T_max, d_T_dec, d_flags);
  if (rc) return rc;
  rc = check_rule(m_max, u);
  if (rc) return rc;
  if (!resident_ok(L)) return fail_with(MPD_ERR_L, "L=%d unsupported for explicit errors (3..128)", L);
  if (n == 0) return MPD_OK;
  if (d_links == nullptr || ((uintptr_t)d_links & 3u)) return fail_with(MPD_ERR_PTR, "links NULL or misaligned");
  if (u > 0 && (d_move_seeds == nullptr || ((uintptr_t)d_move_seeds & 7u)))
    return fail_with(MPD_ERR_PTR, "random moves need aligned move seeds");
  ResidentArgs a = {};
  a.L = L;
  a.n = n;
  a.links = d_links;
  a.T_max = T_max;
  a.t_exact = -1;
  a.T_dec = d_T_dec;
  a.flags = d_flags;
  a.syn = d_final_syndrome;
  a.m_max = m_max;
  a.u = u;
  a.move_seeds = d_move_seeds;
  a.open = open;
  if (open && !open_ok(L)) return fail_with(MPD_ERR_L, "L=%d unsupported on the open lattice (3..128)", L);
  return launch_resident(a, (hipStream_t)stream);
}

static int run_steps_rule(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n, int t_exact,
                          int m_max, int u, int16_t *d_m_out, uint32_t *d_sigma_out, uint8_t *d_wind_out,
                          void *stream, int open = 0);

int mpd_decode_errors(int L, const uint32_t *d_links, int64_t n, int T_max, int32_t *d_T_dec, uint8_t *d_flags,
                      uint32_t *d_final_syndrome, void *d_workspace, size_t ws_bytes, void *stream) {
  g_last_error.clear();
  if (resident_ok(L) || !tiled_ok(L))
    return decode_links_rule(L, d_links, nullptr, n, T_max, 0, 0, d_T_dec, d_flags, d_final_syndrome, stream);
  // the band path (L >= 256): the same passes as a seeded decode
  int rc = check_common(L, n, T_max, d_T_dec, d_flags);
  if (rc) return rc;
  if (n == 0) return MPD_OK;
  if (n > BAND_MAX_N) return fail_with(MPD_ERR_N, "n=%lld: at most %d samples per band-path call", (long long)n, BAND_MAX_N);
  if (d_links == nullptr || ((uintptr_t)d_links & 3u)) return fail_with(MPD_ERR_PTR, "links NULL or misaligned");
  if (d_final_syndrome != nullptr && ((uintptr_t)d_final_syndrome & 3u))
    return fail_with(MPD_ERR_PTR, "final_syndrome misaligned");
  const size_t need = mpd_workspace_bytes(L, n);
  if (ws_bytes < need || d_workspace == nullptr)
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
  if ((uintptr_t)d_workspace & 255u) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  BandRun r;
  rc = band_setup(r, L, 0, nullptr, nullptr, n, T_max, d_T_dec, d_flags, d_final_syndrome, d_workspace,
                  (hipStream_t)stream, d_links);
  if (rc != MPD_OK) return rc;
  return band_passes(&r, 1);
}

// Band-path state export and resume: exactly t_exact steps after t_start,
// from explicit errors (m_in == nullptr) or from an exported state.
static int band_steps_export(int L, const uint32_t *d_links, const int16_t *d_m_in, const uint32_t *d_sigma_in,
                             const uint8_t *d_wind_in, int64_t n, int t_start, int t_exact, int m_max, int u,
                             const uint64_t *d_move_seeds, int16_t *d_m_out, uint32_t *d_sigma_out,
                             uint8_t *d_wind_out, void *d_workspace, size_t ws_bytes, hipStream_t st) {
  if (n > BAND_MAX_N) return fail_with(MPD_ERR_N, "n=%lld: at most %d samples per band-path call", (long long)n, BAND_MAX_N);
  const size_t need = mpd_workspace_bytes(L, n);
  if (ws_bytes < need || d_workspace == nullptr)
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
  if ((uintptr_t)d_workspace & 255u) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  const BandWorkspace w = band_layout(L, n, d_workspace);
  Rule rule;
  rule.m_max = m_max;
  rule.u = u;
  rule.seeds = d_move_seeds;
  const int P = L / 2, NJ = L / TILE_H;
  const int64_t strips = n * NJ * P;
  hipLaunchKernelGGL(k_tile_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, w.alive, w.wind, w.status,
                     w.t_done, w.active[0], &w.count[2]);
  HIP_TRY(hipGetLastError());
  if (d_m_in == nullptr) {
    hipLaunchKernelGGL(k_band_links, dim3((unsigned)((strips + 255) / 256)), dim3(256), 0, st, L, n, d_links, w.S[0],
                       w.wind);
  } else {
    hipLaunchKernelGGL(k_band_state_import, dim3((unsigned)((strips + 255) / 256)), dim3(256), 0, st, L, n, t_start,
                       d_m_in, d_sigma_in, d_wind_in, w.E[0], w.S[0], w.wind, w.t_done);
  }
  HIP_TRY(hipGetLastError());
  int buf = 0;
  int rc = band_run_exact(L, n, t_start, t_exact, w, rule, st, &buf);
  if (rc != MPD_OK) return rc;
  const int64_t words = n * ((int64_t)L * L / 32);
  hipLaunchKernelGGL(k_band_state_export, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, L, n,
                     t_start + t_exact, m_max, w.E[buf], w.S[buf], w.wind, d_m_out, d_sigma_out, d_wind_out);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

int mpd_run_steps_ws(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n, int t_exact, int m_max,
                     int u, int16_t *d_m_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *d_workspace,
                     size_t ws_bytes, void *stream) {
  g_last_error.clear();
  if (resident_ok(L) || !tiled_ok(L))
    return run_steps_rule(L, d_links, d_move_seeds, n, t_exact, m_max, u, d_m_out, d_sigma_out, d_wind_out, stream);
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "n out of range");
  if (t_exact < 0 || t_exact > MPD_T_MAX_LIMIT) return fail_with(MPD_ERR_TMAX, "t_exact out of range");
  const int rc = check_rule(m_max, u);
  if (rc) return rc;
  if (n == 0) return MPD_OK;
  if (d_links == nullptr || ((uintptr_t)d_links & 3u)) return fail_with(MPD_ERR_PTR, "links NULL or misaligned");
  if (d_m_out == nullptr || d_sigma_out == nullptr || d_wind_out == nullptr || ((uintptr_t)d_m_out & 1u) ||
      ((uintptr_t)d_sigma_out & 3u))
    return fail_with(MPD_ERR_PTR, "state outputs NULL or misaligned");
  if (u > 0 && (d_move_seeds == nullptr || ((uintptr_t)d_move_seeds & 7u)))
    return fail_with(MPD_ERR_PTR, "random moves need aligned move seeds");
  return band_steps_export(L, d_links, nullptr, nullptr, nullptr, n, 0, t_exact, m_max, u, d_move_seeds, d_m_out,
                           d_sigma_out, d_wind_out, d_workspace, ws_bytes, (hipStream_t)stream);
}

int mpd_run_steps_from_ws(int L, const int16_t *d_m_in, const uint32_t *d_sigma_in, const uint8_t *d_wind_in,
                          int64_t n, int t_start, int t_exact, int m_max, int u, const uint64_t *d_move_seeds,
                          int16_t *d_m_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *d_workspace,
                          size_t ws_bytes, void *stream) {
  g_last_error.clear();
  if (resident_ok(L) || !tiled_ok(L))
    return mpd_run_steps_from(L, d_m_in, d_sigma_in, d_wind_in, n, t_start, t_exact, m_max, u, d_move_seeds, d_m_out,
                              d_sigma_out, d_wind_out, stream);
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "n out of range");
  if (t_start < 0 || t_exact < 0 || (int64_t)t_start + t_exact > MPD_T_MAX_LIMIT)
    return fail_with(MPD_ERR_TMAX, "t_start=%d, t_exact=%d: both >= 0 with a sum <= %d", t_start, t_exact,
                     MPD_T_MAX_LIMIT);
  const int rc = check_rule(m_max, u);
  if (rc) return rc;
  if (n == 0) return MPD_OK;
  if (d_m_in == nullptr || d_sigma_in == nullptr || d_wind_in == nullptr || ((uintptr_t)d_m_in & 1u) ||
      ((uintptr_t)d_sigma_in & 3u))
    return fail_with(MPD_ERR_PTR, "state inputs NULL or misaligned");
  if (d_m_out == nullptr || d_sigma_out == nullptr || d_wind_out == nullptr || ((uintptr_t)d_m_out & 1u) ||
      ((uintptr_t)d_sigma_out & 3u))
    return fail_with(MPD_ERR_PTR, "state outputs NULL or misaligned");
  if (u > 0 && (d_move_seeds == nullptr || ((uintptr_t)d_move_seeds & 7u)))
    return fail_with(MPD_ERR_PTR, "random moves need aligned move seeds");
  return band_steps_export(L, nullptr, d_m_in, d_sigma_in, d_wind_in, n, t_start, t_exact, m_max, u, d_move_seeds,
                           d_m_out, d_sigma_out, d_wind_out, d_workspace, ws_bytes, (hipStream_t)stream);
}

int mpd_decode_errors_rule(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n, int T_max,
                           int m_max, int u, int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_final_syndrome,
                           void *stream) {
  g_last_error.clear();
  return decode_links_rule(L, d_links, d_move_seeds, n, T_max, m_max, u, d_T_dec, d_flags, d_final_syndrome, stream);
}

static int run_steps_rule(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n, int t_exact, int m_max,
                   int u, int16_t *d_m_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream, int open) {
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "n out of range");
  if (t_exact < 0 || t_exact > MPD_T_MAX_LIMIT) return fail_with(MPD_ERR_TMAX, "t_exact out of range");
  const int rc = check_rule(m_max, u);
  if (rc) return rc;
  if (!resident_ok(L)) return fail_with(MPD_ERR_L, "L=%d unsupported for run_steps (3..128)", L);
  if (n == 0) return MPD_OK;
  if (d_links == nullptr || ((uintptr_t)d_links & 3u)) return fail_with(MPD_ERR_PTR, "links NULL or misaligned");
  if (d_m_out == nullptr || d_sigma_out == nullptr || d_wind_out == nullptr)
    return fail_with(MPD_ERR_PTR, "state outputs must not be NULL");
  if (u > 0 && (d_move_seeds == nullptr || ((uintptr_t)d_move_seeds & 7u)))
    return fail_with(MPD_ERR_PTR, "random moves need aligned move seeds");
  ResidentArgs a = {};
  a.L = L;
  a.n = n;
  a.links = d_links;
  a.T_max = t_exact;
  a.t_exact = t_exact;
  a.syn = d_sigma_out;
  a.m_out = d_m_out;
  a.wind_out = d_wind_out;
  a.m_max = m_max;
  a.u = u;
  a.move_seeds = d_move_seeds;
  a.open = open;
  if (open && !open_ok(L)) return fail_with(MPD_ERR_L, "L=%d unsupported on the open lattice (3..128)", L);
  return launch_resident(a, (hipStream_t)stream);
}

int mpd_run_steps_from(int L, const int16_t *d_m_in, const uint32_t *d_sigma_in, const uint8_t *d_wind_in, int64_t n,
                       int t_start, int t_exact, int m_max, int u, const uint64_t *d_move_seeds, int16_t *d_m_out,
                       uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream) {
  g_last_error.clear();
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "n out of range");
  if (t_start < 0 || t_exact < 0 || (int64_t)t_start + t_exact > MPD_T_MAX_LIMIT)
    return fail_with(MPD_ERR_TMAX, "t_start=%d, t_exact=%d: both >= 0 with a sum <= %d", t_start, t_exact,
                     MPD_T_MAX_LIMIT);
  const int rc = check_rule(m_max, u);
  if (rc) return rc;
  if (!resident_ok(L)) return fail_with(MPD_ERR_L, "L=%d unsupported for run_steps_from (3..128)", L);
  if (n == 0) return MPD_OK;
  if (d_m_in == nullptr || d_sigma_in == nullptr || d_wind_in == nullptr || ((uintptr_t)d_m_in & 1u) ||
      ((uintptr_t)d_sigma_in & 3u))
    return fail_with(MPD_ERR_PTR, "state inputs NULL or misaligned");
  if (d_m_out == nullptr || d_sigma_out == nullptr || d_wind_out == nullptr || ((uintptr_t)d_m_out & 1u) ||
      ((uintptr_t)d_sigma_out & 3u))
    return fail_with(MPD_ERR_PTR, "state outputs NULL or misaligned");
  if (u > 0 && (d_move_seeds == nullptr || ((uintptr_t)d_move_seeds & 7u)))
    return fail_with(MPD_ERR_PTR, "random moves need aligned move seeds");
  ResidentArgs a = {};
  a.L = L;
  a.n = n;
  a.T_max = t_exact;
  a.t_exact = t_exact;
  a.syn = d_sigma_out;
  a.m_out = d_m_out;
  a.wind_out = d_wind_out;
  a.m_max = m_max;
  a.u = u;
  a.move_seeds = d_move_seeds;
  a.m_in = d_m_in;
  a.syn_in = d_sigma_in;
  a.wind_in = d_wind_in;
  a.t_start = t_start;
  return launch_resident(a, (hipStream_t)stream);
}

int mpd_run_steps(int L, const uint32_t *d_links, int64_t n, int t_exact, int16_t *d_m_out, uint32_t *d_sigma_out,
                  uint8_t *d_wind_out, void *stream) {
  g_last_error.clear();
  return run_steps_rule(L, d_links, nullptr, n, t_exact, 0, 0, d_m_out, d_sigma_out, d_wind_out, stream);
}

int mpd_run_steps_rule(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n, int t_exact,
                       int m_max, int u, int16_t *d_m_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream) {
  g_last_error.clear();
  return run_steps_rule(L, d_links, d_move_seeds, n, t_exact, m_max, u, d_m_out, d_sigma_out, d_wind_out, stream);
}


// ---------------------------------------------------------------------------
// Open lattice (rough left / right boundaries), resident kernel only
// ---------------------------------------------------------------------------

int mpd_decode_open(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int32_t *d_T_dec,
                    uint8_t *d_flags, uint32_t *d_final_syndrome, void *d_workspace, size_t ws_bytes, void *stream) {
  g_last_error.clear();
  if (!(p >= 0.0 && p <= 1.0)) return fail_with(MPD_ERR_P, "p must lie in [0, 1]");
  const int rc = check_common(L, n, T_max, d_T_dec, d_flags);
  if (rc) return rc;
  if (!open_ok(L) && !tiled_ok(L))
    return fail_with(MPD_ERR_L, "L=%d unsupported on the open lattice (3..128, or a multiple of 16 in [256, 16384])",
                     L);
  if (n == 0) return MPD_OK;
  if (d_seeds == nullptr || ((uintptr_t)d_seeds & 7u)) return fail_with(MPD_ERR_PTR, "seeds NULL or misaligned");
  if (d_final_syndrome != nullptr && ((uintptr_t)d_final_syndrome & 3u))
    return fail_with(MPD_ERR_PTR, "final_syndrome misaligned");
  hipStream_t st = (hipStream_t)stream;
  if (open_ok(L)) {
    ResidentArgs a = {};
    a.L = L;
    a.n = n;
    a.seeds = d_seeds;
    a.thr = threshold_of(p);
    a.T_max = T_max;
    a.t_exact = -1;
    a.T_dec = d_T_dec;
    a.flags = d_flags;
    a.syn = d_final_syndrome;
    a.open = 1;
    return launch_resident(a, st);
  }
  if (n > BAND_MAX_N) return fail_with(MPD_ERR_N, "n=%lld: at most %d samples per band-path call", (long long)n, BAND_MAX_N);
  const size_t need = mpd_workspace_bytes(L, n);
  if (ws_bytes < need || d_workspace == nullptr)
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
  if ((uintptr_t)d_workspace & 255u) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  Rule rule;
  rule.open = true;
  return decode_band(L, threshold_of(p), nullptr, d_seeds, n, T_max, d_T_dec, d_flags, d_final_syndrome, d_workspace,
                     rule, st);
}

int mpd_decode_errors_open(int L, const uint32_t *d_links, int64_t n, int T_max, int32_t *d_T_dec, uint8_t *d_flags,
                           uint32_t *d_final_syndrome, void *stream) {
  g_last_error.clear();
  return decode_links_rule(L, d_links, nullptr, n, T_max, 0, 0, d_T_dec, d_flags, d_final_syndrome, stream, 1);
}

int mpd_run_steps_open(int L, const uint32_t *d_links, int64_t n, int t_exact, int16_t *d_m_out,
                       uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream) {
  g_last_error.clear();
  return run_steps_rule(L, d_links, nullptr, n, t_exact, 0, 0, d_m_out, d_sigma_out, d_wind_out, stream, 1);
}

}  // extern "C"
