// async.hip -- desynchronized decoders on the GPU (Sec. "Desynchronization
// and Lindbladian dynamics": Def. "simulation and lag times", Def. "marching
// soldiers desynchronization", Def. "desynchronized decoders"; Sec.
// "Uncoordinated desynchronization").
//
// Marching soldiers.  Every site runs the synchronous schedule at its own
// pace: v = 3 message updates, then one feedback update that applies F to the
// two links the site owns (r -> r + x-hat, r -> r + y-hat); t_sim counts
// these updates.  An update of r is accepted only if no site within
// infinity-distance 2 (twice the range Delta = 1 over which A and F read and
// write) is behind r.  A site keeps m^old and m^new: a neighbour one update
// ahead shows m^old, a level one m^new.  Feedback of step k must see each
// syndrome before any step-k feedback: the flips applied at a site by step-k
// feedback are recorded in a flip parity of slot k mod 2, which the reader
// undoes; a site clears the slot of step k - 1 when it starts step k.  The
// simulated dynamics is then exactly the synchronous decoder's, whatever the
// order of the accepted updates (Prop. "faithful Lindbladian simulation").
//
// Uncoordinated (template mode UNC).  The same clock and rounds without the
// lag rule or old copies: message updates read current values, and a motion
// update moves the site's anyon along its force (uncoord_update).
//
// Clock: time runs in slots.  In slot s site i rings iff word 2(i&1) of
// Philox4x32-10(key = seed, counter (i >> 1, s, CLOCK_TAG, 0)) is below the
// ring threshold, and the ringing sites attempt one update each in
// increasing order of (word 2(i&1)+1 >> 13, i).  The workgroup realises that
// order in parallel rounds: every pending ringer whose key is the smallest
// among the pending ringers within distance 2 attempts.  Those sites are more than
// 2 apart, so what they read and write is disjoint; updates more than 2
// apart commute; and any two ringers within distance 2 attempt in key order.
// Each slot therefore ends in the state of the sequential order.
//
// A ringer's key is (priority word >> 13) << 13 | i, unique per site (i <
// 4096); the largest, 0xFFFFEFFF, stays below the key ~0 of an idle site (not
// ringing, or done for this slot).  A pending site is ready when its key is
// the minimum of the 5 x 5 box around it.  Only pending sites are visited:
// they are kept in a list (the ringers at the start of a slot, then the ones
// not ready in a round), so a round reads the 25 keys of each pending site's
// box instead of two passes over every site.
//
// One workgroup holds one sample (5 <= L <= 64) in LDS for its whole run:
//   K       u32 per site: key of the current slot
//   PL      two u16 lists of the pending sites (the current round's, the next)
//   MN, MO  uint2 per site: m^new / m^old in distance form, packed u16
//           (.x = m^{+x} | m^{-x} << 16, .y = m^{+y} | m^{-y} << 16)
//   TS      u16 simulation time
//   FL      u8: bit 0 anyon (the physical syndrome), bit 1 + (k & 1) flip
//           parity of step k
//   CH      u8: bit 0 x-link, bit 1 y-link of the correction chain (during
//           set-up: of the error chain)
//   RL      u16 list of the sites ready in the current round, so that the
//           updates run on consecutive lanes instead of scattered ones
// Registers and t_sim stay below 2^16 because at most one update per site
// happens per slot and the slot count is capped.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "engine.h"
#include "host.h"
#include "mpd.h"

namespace mpd {

constexpr uint32_t CLOCK_TAG = 0x41535943u;
constexpr uint32_t TYPE_TAG = 0x54595045u;   // update type of the uncoordinated "random" schedule

struct AsyncArgs {
  int L;
  const uint64_t *seeds;   // per sample: noise key (seeded mode) and clock key
  uint64_t thr;            // noise flip threshold (seeded mode)
  const uint32_t *links;   // explicit error chains, or nullptr for seeded noise
  uint64_t ring_thr;       // ring probability per slot times 2^32, in [1, 2^32]
  int t_target;            // >= 0: run until every site has made 4 t_target updates
  int S_max;               // slot budget
  int sched;               // uncoordinated schedule: 0 cyclic, 1 random update types
  int32_t *T_async;
  uint8_t *flags;
  int32_t *slots;
  int64_t *updates;
  uint32_t *syn;
  int16_t *m_out;
  uint16_t *tsim_out;
  uint8_t *wind_out;
};

constexpr uint32_t IDLE = 0xFFFFFFFFu;
constexpr int ASYNC_SITES = 4;   // sites per thread; the launch uses at least N / 4 threads

size_t async_lds(int L) {
  const size_t N = (size_t)L * L;
  return ((30 * N + 15) & ~(size_t)15) + 64;
}



__device__ __forceinline__ int wrapc(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// A^{(D)} for one register: 1 if an anyon sits on the line, else the
// smallest nonzero register on it plus one, else 0.  A register minus one
// taken mod 2^16 maps 0 ("no message") above every live value.
__device__ __forceinline__ uint32_t rule_A(bool anyon, uint32_t a, uint32_t b, uint32_t c) {
  if (anyon) return 1u;
  const uint32_t t = min(min((a - 1u) & 0xFFFFu, (b - 1u) & 0xFFFFu), (c - 1u) & 0xFFFFu);
  return t == 0xFFFFu ? 0u : t + 2u;
}

// sgn(m^{-a} - m^{+a}) with an absent message counted as +infinity.
__device__ __forceinline__ int force_of(uint32_t mp, uint32_t mm) {
  if (mp == 0u && mm == 0u) return 0;
  if (mp == 0u) return -1;
  if (mm == 0u) return 1;
  return (mm > mp) - (mm < mp);
}

// Forces of an anyon site from its registers: argmin' over the nonzero
// registers, ties ordered -y, -x, +x, +y (eq. (degbreak)); the force acts
// along the winning axis only.
__device__ __forceinline__ void site_force(uint2 m, int &fx, int &fy) {
  const uint32_t px = m.x & 0xFFFFu, mx = m.x >> 16, py = m.y & 0xFFFFu, my = m.y >> 16;
  uint32_t best = 0xFFFFFFFFu;
  int axis = -1;
  if (my && my * 4u + 0u < best) { best = my * 4u + 0u; axis = 1; }
  if (mx && mx * 4u + 1u < best) { best = mx * 4u + 1u; axis = 0; }
  if (px && px * 4u + 2u < best) { best = px * 4u + 2u; axis = 0; }
  if (py && py * 4u + 3u < best) { best = py * 4u + 3u; axis = 1; }
  fx = axis == 0 ? force_of(px, mx) : 0;
  fy = axis == 1 ? force_of(py, my) : 0;
}

// Workgroup OR of a predicate through a single barrier (the library form
// takes three).  Three flags rotate: call c ORs into flag c % 3 and clears
// flag (c + 1) % 3 for the next call, before its barrier.  The readers of a
// flag read it right after the barrier of its call and pass one more barrier
// before the flag is cleared again, and the next writers of the cleared flag
// start only after this call's barrier.  Every thread must make the same
// calls.
__device__ __forceinline__ bool wg_or(bool pred, int *flags, uint32_t &c) {
  const uint32_t cur = c % 3u, nxt = (c + 1u) % 3u;
  ++c;
  if (threadIdx.x == 0) flags[nxt] = 0;
  if (__ballot(pred) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&flags[cur], 1);
  __syncthreads();
  return flags[cur] != 0;
}

struct AsyncLds {
  uint32_t *K;
  uint16_t *PL[2];
  uint2 *MN, *MO;
  uint16_t *TS;
  uint8_t *FL, *CH;
  uint16_t *RL;
};

// One attempted update of site i.  Returns 0 if rejected, 1 if accepted,
// 2 if accepted and a link flipped.
__device__ __forceinline__ int async_attempt(const AsyncLds &s, int L, int i, int x, int y) {
  int col[5], row[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    col[d] = wrapc(x + d - 2, L);
    row[d] = wrapc(y + d - 2, L) * L;
  }
  // every t_sim of the 5 x 5 ball, loaded together
  uint32_t tv[5][5];
#pragma unroll
  for (int dy = 0; dy < 5; ++dy)
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) tv[dy][dx] = s.TS[row[dy] + col[dx]];
  const uint32_t j = tv[2][2];
  uint32_t tmin = 0xFFFFu;
#pragma unroll
  for (int dy = 0; dy < 5; ++dy)
#pragma unroll
    for (int dx = 0; dx < 5; ++dx)
      if (dx != 2 || dy != 2) tmin = min(tmin, tv[dy][dx]);
  if (tmin < j) return 0;
  const int xl = col[1], xr = col[3];
  const int rd = row[1], rc = row[2], ru = row[3];
  const uint32_t k = j >> 2, phase = j & 3u;
  int ret = 1;
  if (phase < 3u) {
    // present views of the 3 x 3 block: level neighbours show m^new, those
    // one update ahead m^old
    auto an = [&](int q) { return (s.FL[q] & 1u) != 0u; };
    const int dl = rd + xl, dc = rd + x, dr = rd + xr;
    const int cl = rc + xl, cr = rc + xr;
    const int ul = ru + xl, uc = ru + x, ur = ru + xr;
    const uint2 mdl = (tv[1][1] == j ? s.MN : s.MO)[dl], mdc = (tv[1][2] == j ? s.MN : s.MO)[dc],
                mdr = (tv[1][3] == j ? s.MN : s.MO)[dr], mcl = (tv[2][1] == j ? s.MN : s.MO)[cl],
                mcr = (tv[2][3] == j ? s.MN : s.MO)[cr], mul = (tv[3][1] == j ? s.MN : s.MO)[ul],
                muc = (tv[3][2] == j ? s.MN : s.MO)[uc], mur = (tv[3][3] == j ? s.MN : s.MO)[ur];
    const uint32_t px = rule_A(an(dl) || an(cl) || an(ul), mdl.x & 0xFFFFu, mcl.x & 0xFFFFu, mul.x & 0xFFFFu);
    const uint32_t mx = rule_A(an(dr) || an(cr) || an(ur), mdr.x >> 16, mcr.x >> 16, mur.x >> 16);
    const uint32_t py = rule_A(an(dl) || an(dc) || an(dr), mdl.y & 0xFFFFu, mdc.y & 0xFFFFu, mdr.y & 0xFFFFu);
    const uint32_t my = rule_A(an(ul) || an(uc) || an(ur), mul.y >> 16, muc.y >> 16, mur.y >> 16);
    if (phase == 0u && k > 0u) s.FL[i] = (uint8_t)(s.FL[i] & ~(2u << ((k - 1u) & 1u)));
    s.MO[i] = s.MN[i];
    s.MN[i] = make_uint2(px | mx << 16, py | my << 16);
  } else {
    // feedback of step k on the links r -> r + x-hat and r -> r + y-hat
    const uint32_t sb = 2u << (k & 1u);
    const int ix = rc + xr, iy = ru + x;
    auto an = [&](int q) { return ((s.FL[q] ^ ((s.FL[q] & sb) ? 1u : 0u)) & 1u) != 0u; };
    const bool ar = an(i), ax = an(ix), ay = an(iy);
    const uint2 vr = s.MN[i], vx = (tv[2][3] == j ? s.MN : s.MO)[ix], vy = (tv[3][2] == j ? s.MN : s.MO)[iy];
    int fxr = 0, fyr = 0, fxx = 0, fyx = 0, fxy = 0, fyy = 0;
    if (ar) site_force(vr, fxr, fyr);
    if (ax) site_force(vx, fxx, fyx);
    if (ay) site_force(vy, fxy, fyy);
    // link exponent sigma_r f_r OR sigma_{r+a} (-f_{r+a}); f = 0 off anyons
    const bool lx = (ar && fxr == -1) || (ax && fxx == 1);
    const bool ly = (ar && fyr == -1) || (ay && fyy == 1);
    const uint32_t t = 1u | sb;
    if (lx) {
      s.CH[i] ^= 1u;
      s.FL[i] ^= t;
      s.FL[ix] ^= t;
    }
    if (ly) {
      s.CH[i] ^= 2u;
      s.FL[i] ^= t;
      s.FL[iy] ^= t;
    }
    if (lx || ly) ret = 2;
    s.MO[i] = s.MN[i];
  }
  s.TS[i] = (uint16_t)(j + 1u);
  return ret;
}

// One update of site i of the uncoordinated desynchronization: no lag rule
// and no old copies.  Message updates read the current registers and anyon
// bits on their lines; a motion update of an anyon site moves its anyon one
// link along its force (+a for f^a = -1, -a for f^a = +1), annihilating it
// with an anyon there.  Schedule 0: every fourth update of a site is a
// motion; schedule 1: an update is a motion iff word (i & 1) of
// Philox(key, counter (i >> 1, slot, TYPE_TAG, 0)) mod 4 is 3.  Returns 1, or
// 2 if a link flipped.
__device__ __forceinline__ int uncoord_update(const AsyncLds &s, int L, int i, int x, int y, int sched,
                                              uint32_t slot, uint32_t k0, uint32_t k1) {
  const uint32_t j = s.TS[i];
  bool motion;
  if (sched == 0) {
    motion = (j & 3u) == 3u;
  } else {
    const Words4 w = philox4x32_10((uint32_t)i >> 1, k0, k1, slot, TYPE_TAG);
    motion = (((i & 1) ? w.w1 : w.w0) & 3u) == 3u;
  }
  const int xl = wrapc(x - 1, L), xr = wrapc(x + 1, L);
  const int rd = wrapc(y - 1, L) * L, rc = y * L, ru = wrapc(y + 1, L) * L;
  int ret = 1;
  if (!motion) {
    auto an = [&](int q) { return (s.FL[q] & 1u) != 0u; };
    const int dl = rd + xl, dc = rd + x, dr = rd + xr;
    const int cl = rc + xl, cr = rc + xr;
    const int ul = ru + xl, uc = ru + x, ur = ru + xr;
    const uint2 mdl = s.MN[dl], mdc = s.MN[dc], mdr = s.MN[dr], mcl = s.MN[cl], mcr = s.MN[cr], mul = s.MN[ul],
                muc = s.MN[uc], mur = s.MN[ur];
    const uint32_t px = rule_A(an(dl) || an(cl) || an(ul), mdl.x & 0xFFFFu, mcl.x & 0xFFFFu, mul.x & 0xFFFFu);
    const uint32_t mx = rule_A(an(dr) || an(cr) || an(ur), mdr.x >> 16, mcr.x >> 16, mur.x >> 16);
    const uint32_t py = rule_A(an(dl) || an(dc) || an(dr), mdl.y & 0xFFFFu, mdc.y & 0xFFFFu, mdr.y & 0xFFFFu);
    const uint32_t my = rule_A(an(ul) || an(uc) || an(ur), mul.y >> 16, muc.y >> 16, mur.y >> 16);
    s.MN[i] = make_uint2(px | mx << 16, py | my << 16);
  } else if (s.FL[i] & 1u) {
    int fx, fy;
    site_force(s.MN[i], fx, fy);
    int q = -1;
    if (fx == -1) {
      q = rc + xr;
      s.CH[i] ^= 1u;
    } else if (fx == 1) {
      q = rc + xl;
      s.CH[q] ^= 1u;
    } else if (fy == -1) {
      q = ru + x;
      s.CH[i] ^= 2u;
    } else if (fy == 1) {
      q = rd + x;
      s.CH[q] ^= 2u;
    }
    if (q >= 0) {
      s.FL[i] ^= 1u;
      s.FL[q] ^= 1u;
      ret = 2;
    }
  }
  s.TS[i] = (uint16_t)(j + 1u);
  return ret;
}

// UNC selects the uncoordinated desynchronization; the clock, the rounds and
// the outputs are shared (its ready sites are likewise more than 2 apart,
// and what it reads and writes lies within distance 1).
template <bool UNC>
__global__ __launch_bounds__(1024) void k_async(AsyncArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int L = a.L, N = L * L;
  AsyncLds s;
  s.K = (uint32_t *)lds;
  s.PL[0] = (uint16_t *)(s.K + N);
  s.PL[1] = s.PL[0] + N;
  s.MN = (uint2 *)(s.PL[1] + N);
  s.MO = s.MN + N;
  s.TS = (uint16_t *)(s.MO + N);
  s.FL = (uint8_t *)(s.TS + N);
  s.CH = s.FL + N;
  s.RL = (uint16_t *)(s.CH + N);
  // wind bits, 1 + last flip slot, updates, lengths of the ready list (two),
  // the three flags of wg_or, lengths of the pending lists (two)
  int *RED = (int *)(lds + ((30 * (size_t)N + 15) & ~(size_t)15));
  int *RC = RED + 3, *PC = RED + 8;
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, T = blockDim.x;
  const uint64_t seed = a.seeds != nullptr ? a.seeds[b] : 0u;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (tid < 16) RED[tid] = 0;
  const int LW = (2 * N + 31) / 32;
  for (int i = tid; i < N; i += T) {
    uint32_t e;
    if (a.links != nullptr) {
      const uint32_t w = a.links[b * LW + ((2 * i) >> 5)];
      e = (w >> ((2 * i) & 31)) & 3u;
    } else {
      bool fx, fy;
      site_noise((uint32_t)i, k0, k1, a.thr, fx, fy);
      e = (fx ? 1u : 0u) | (fy ? 2u : 0u);
    }
    s.CH[i] = (uint8_t)e;
    s.MN[i] = make_uint2(0u, 0u);
    s.MO[i] = make_uint2(0u, 0u);
    s.TS[i] = 0;
  }
  __syncthreads();
  uint32_t wind = 0;
  for (int i = tid; i < N; i += T) {
    const int x = i % L, y = i / L;
    const uint32_t e = s.CH[i];
    const uint32_t par = (e ^ s.CH[y * L + wrapc(x - 1, L)] ^ (e >> 1) ^ (s.CH[wrapc(y - 1, L) * L + x] >> 1)) & 1u;
    s.FL[i] = (uint8_t)par;
    if (x == L - 1) wind ^= e & 1u;
    if (y == L - 1) wind ^= e & 2u;
  }
  if (wind) atomicXor(&RED[0], (int)wind);
  __syncthreads();
  for (int i = tid; i < N; i += T) s.CH[i] = 0;
  __syncthreads();

  const bool run = a.t_target >= 0;
  const uint32_t target = run ? 4u * (uint32_t)a.t_target : 0u;
  int last_flip = -1;
  uint32_t my_updates = 0;
  int slot = 0;
  int busy_any = 0;
  uint32_t orc = 0;  // calls of wg_or so far (RED[5..7] are its flags)
  for (;; ++slot) {
    int busy = 0;
    for (int i = tid; i < N; i += T) busy |= run ? (s.TS[i] < target) : (s.FL[i] != 0);
    if (tid == 0) {  // read by every thread before the last barrier of the previous slot
      RC[0] = 0;
      RC[1] = 0;
    }
    if (slot < a.S_max) {
      // ring draws; the ringers are listed as the pending sites of round 0
      // (PC[0] is zero here: its last round ended on an empty list, or zeroed it)
      const int lane = tid & 63;
      const uint64_t below = (lane ? (~0ull >> (64 - lane)) : 0ull);
      for (int h0 = 0; 2 * h0 < N; h0 += T) {
        const int h = h0 + tid;
        const int i0 = 2 * h, i1 = 2 * h + 1;
        bool r0 = false, r1 = false;
        if (2 * h < N) {
          const Words4 w = philox4x32_10((uint32_t)h, k0, k1, (uint32_t)slot, CLOCK_TAG);
          r0 = (uint64_t)w.w0 < a.ring_thr && (!run || s.TS[i0] < target);
          s.K[i0] = r0 ? ((w.w1 >> 13) << 13 | (uint32_t)i0) : IDLE;
          if (i1 < N) {
            r1 = (uint64_t)w.w2 < a.ring_thr && (!run || s.TS[i1] < target);
            s.K[i1] = r1 ? ((w.w3 >> 13) << 13 | (uint32_t)i1) : IDLE;
          }
        }
        const uint64_t b0 = __ballot(r0), b1 = __ballot(r1);
        const int tot = __popcll(b0) + __popcll(b1);
        if (tot) {
          int base = 0;
          if (lane == 0) base = atomicAdd(&PC[0], tot);
          base = __builtin_amdgcn_readfirstlane(base);
          if (r0) s.PL[0][base + __popcll(b0 & below)] = (uint16_t)i0;
          if (r1) s.PL[0][base + __popcll(b0) + __popcll(b1 & below)] = (uint16_t)i1;
        }
      }
    }
    busy_any = wg_or(busy != 0, RED + 5, orc);
    if (!busy_any || slot >= a.S_max) break;
    // Rounds.  Phase A: every pending site reads the keys of its 5 x 5 box
    // (a snapshot: no key changes in this phase); the box minimum is ready
    // and goes to the ready list, the others to the next pending list.
    // Phase B: the ready sites go idle and attempt their updates.  Counters
    // alternate between rounds, each cleared by thread 0 once every thread
    // has read it (after the barrier that follows its last read).
    for (int cur = 0;; cur ^= 1) {
      const int npend = PC[cur];
      if (npend == 0) break;
      const int nxt = cur ^ 1;
      // the lists by select, not by indexing (an indexed array would live in
      // private memory)
      const uint16_t *plc = cur ? s.PL[1] : s.PL[0];
      uint16_t *pln = cur ? s.PL[0] : s.PL[1];
      const int lane = tid & 63;
      const uint64_t below = (lane ? (~0ull >> (64 - lane)) : 0ull);
      for (int e0 = 0; e0 < npend; e0 += T) {
        const int e = e0 + tid;
        bool ready = false, keep = false;
        int i = 0;
        if (e < npend) {
          i = plc[e];
          const int x = i % L, y = i / L;
          int col[5];
#pragma unroll
          for (int d = 0; d < 5; ++d) col[d] = wrapc(x + d - 2, L);
          uint32_t kb[5][5];
#pragma unroll
          for (int dy = 0; dy < 5; ++dy) {
            const int r0 = wrapc(y + dy - 2, L) * L;
#pragma unroll
            for (int dx = 0; dx < 5; ++dx) kb[dy][dx] = s.K[r0 + col[dx]];
          }
          uint32_t m = IDLE;
#pragma unroll
          for (int dy = 0; dy < 5; ++dy)
#pragma unroll
            for (int dx = 0; dx < 5; ++dx) m = min(m, kb[dy][dx]);
          ready = m == kb[2][2];
          keep = !ready;
        }
        const uint64_t br = __ballot(ready), bk = __ballot(keep);
        int baser = 0, basek = 0;
        if (lane == 0) {
          if (br) baser = atomicAdd(&RC[cur], __popcll(br));
          if (bk) basek = atomicAdd(&PC[nxt], __popcll(bk));
        }
        baser = __builtin_amdgcn_readfirstlane(baser);
        basek = __builtin_amdgcn_readfirstlane(basek);
        if (ready) s.RL[baser + __popcll(br & below)] = (uint16_t)i;
        if (keep) pln[basek + __popcll(bk & below)] = (uint16_t)i;
      }
      __syncthreads();
      const int nready = RC[cur];
      if (tid == 0) {
        PC[cur] = 0;  // read at this round's start, before the barrier above
        RC[nxt] = 0;  // read in the previous round's phase B, before its closing barrier
      }
      for (int e = tid; e < nready; e += T) {
        const int i = s.RL[e];
        s.K[i] = IDLE;
        const int r = UNC ? uncoord_update(s, L, i, i % L, i / L, a.sched, (uint32_t)slot, k0, k1)
                          : async_attempt(s, L, i, i % L, i / L);
        my_updates += r > 0;
        if (r == 2) last_flip = slot;
      }
      __syncthreads();
    }
  }

  uint32_t cw = 0;
  for (int i = tid; i < N; i += T) {
    const int x = i % L, y = i / L;
    if (x == L - 1) cw ^= (s.CH[i] & 1u) << 2;
    if (y == L - 1) cw ^= (s.CH[i] & 2u) << 2;
  }
  if (cw) atomicXor(&RED[0], (int)cw);
  if (my_updates) atomicAdd(&RED[2], (int)my_updates);
  if (last_flip >= 0) atomicMax(&RED[1], last_flip + 1);
  const int NW = (N + 31) / 32;
  if (a.syn != nullptr)
    for (int s0 = tid & ~63; s0 < N; s0 += T) {
      const int i = s0 + (tid & 63);
      const uint64_t bal = __ballot(i < N && (s.FL[i] & 1u));
      if ((tid & 63) == 0) {
        a.syn[b * NW + s0 / 32] = (uint32_t)bal;
        if (s0 / 32 + 1 < NW) a.syn[b * NW + s0 / 32 + 1] = (uint32_t)(bal >> 32);
      }
    }
  if (a.m_out != nullptr)
    for (int i = tid; i < N; i += T) {
      const uint2 m = s.MN[i];
      int16_t *o = a.m_out + b * 4 * N + i;
      o[0] = (int16_t)(m.x & 0xFFFFu);
      o[N] = (int16_t)(m.x >> 16);
      o[2 * N] = (int16_t)(m.y & 0xFFFFu);
      o[3 * N] = (int16_t)(m.y >> 16);
    }
  if (a.tsim_out != nullptr)
    for (int i = tid; i < N; i += T) a.tsim_out[b * N + i] = s.TS[i];
  __syncthreads();
  if (tid == 0) {
    const uint32_t W = (uint32_t)RED[0];
    const bool timeout = busy_any != 0;
    const bool fail = !run && (timeout || ((W ^ (W >> 2)) & 3u) != 0u);
    if (a.T_async) a.T_async[b] = RED[1];
    if (a.flags) a.flags[b] = (uint8_t)((fail ? 1u : 0u) | (timeout ? 2u : 0u));
    if (a.slots) a.slots[b] = slot;
    if (a.updates) a.updates[b] = RED[2];
    if (a.wind_out) a.wind_out[b] = (uint8_t)W;
  }
}

bool async_ok(int L) { return L >= 5 && L <= 64 && async_lds(L) <= 160 * 1024; }

int launch_async(const AsyncArgs &a, int64_t n, bool unc, hipStream_t stream) {
  const int N = a.L * a.L;
  // four sites per thread (one wave for the smallest lattices), so that small
  // lattices leave room for several workgroups per compute unit
  const int threads = std::min(1024, std::max(64, ((N + 3) / 4 + 63) / 64 * 64));
  if (threads * ASYNC_SITES < N) return fail_with(MPD_ERR_L, "L=%d: more than %d sites per thread", a.L, ASYNC_SITES);
  ProfScope ps(unc ? "k_async_unc" : "k_async", stream);
  if (unc)
    hipLaunchKernelGGL(k_async<true>, dim3((unsigned)n), dim3(threads), async_lds(a.L), stream, a);
  else
    hipLaunchKernelGGL(k_async<false>, dim3((unsigned)n), dim3(threads), async_lds(a.L), stream, a);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

}  // namespace mpd

using namespace mpd;

// Common checks of the desynchronized entry points.
static int async_check(int L, int64_t n, double rho, int S_max, uint64_t *ring_thr) {
  if (!async_ok(L)) return fail_with(MPD_ERR_L, "L=%d unsupported for the desynchronized decoder (5..64)", L);
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "n out of range");
  if (!(rho > 0.0 && rho <= 1.0)) return fail_with(MPD_ERR_P, "rho must lie in (0, 1]");
  if (S_max < 0 || S_max > MPD_ASYNC_SLOT_LIMIT)
    return fail_with(MPD_ERR_TMAX, "S_max=%d outside [0, %d]", S_max, MPD_ASYNC_SLOT_LIMIT);
  const uint64_t t = threshold_of(rho);
  *ring_thr = t < 1u ? 1u : t;
  return MPD_OK;
}

static int decode_desync(bool unc, int sched, int L, double p, const uint64_t *d_seeds, int64_t n, double rho,
                         int S_max, int32_t *d_T, uint8_t *d_flags, int32_t *d_slots, int64_t *d_updates,
                         uint32_t *d_final_syndrome, void *stream) {
  uint64_t ring_thr = 0;
  int rc = async_check(L, n, rho, S_max, &ring_thr);
  if (rc) return rc;
  if (!(p >= 0.0 && p <= 1.0)) return fail_with(MPD_ERR_P, "p must lie in [0, 1]");
  if (n == 0) return MPD_OK;
  if (d_seeds == nullptr || ((uintptr_t)d_seeds & 7u)) return fail_with(MPD_ERR_PTR, "seeds NULL or misaligned");
  if (d_T == nullptr || d_flags == nullptr || ((uintptr_t)d_T & 3u))
    return fail_with(MPD_ERR_PTR, "decoding-time / flags output NULL or misaligned");
  if ((d_slots != nullptr && ((uintptr_t)d_slots & 3u)) || (d_updates != nullptr && ((uintptr_t)d_updates & 7u)) ||
      (d_final_syndrome != nullptr && ((uintptr_t)d_final_syndrome & 3u)))
    return fail_with(MPD_ERR_PTR, "optional output misaligned");
  AsyncArgs a = {};
  a.L = L;
  a.seeds = d_seeds;
  a.thr = threshold_of(p);
  a.ring_thr = ring_thr;
  a.t_target = -1;
  a.S_max = S_max;
  a.sched = sched;
  a.T_async = d_T;
  a.flags = d_flags;
  a.slots = d_slots;
  a.updates = d_updates;
  a.syn = d_final_syndrome;
  return launch_async(a, n, unc, (hipStream_t)stream);
}

static int run_desync(bool unc, int sched, int L, const uint32_t *d_links, const uint64_t *d_clock_seeds, int64_t n, int t_target,
                      double rho, int S_max, int32_t *d_slots, int64_t *d_updates, int16_t *d_m_out,
                      uint16_t *d_tsim_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream) {
  uint64_t ring_thr = 0;
  int rc = async_check(L, n, rho, S_max, &ring_thr);
  if (rc) return rc;
  if (t_target < 0 || t_target > MPD_ASYNC_SLOT_LIMIT / 4)
    return fail_with(MPD_ERR_TMAX, "t_target=%d outside [0, %d]", t_target, MPD_ASYNC_SLOT_LIMIT / 4);
  if (n == 0) return MPD_OK;
  if (d_links == nullptr || ((uintptr_t)d_links & 3u)) return fail_with(MPD_ERR_PTR, "links NULL or misaligned");
  if (d_clock_seeds == nullptr || ((uintptr_t)d_clock_seeds & 7u))
    return fail_with(MPD_ERR_PTR, "clock seeds NULL or misaligned");
  if (d_slots == nullptr || d_m_out == nullptr || d_tsim_out == nullptr || d_sigma_out == nullptr ||
      d_wind_out == nullptr || ((uintptr_t)d_slots & 3u) || ((uintptr_t)d_m_out & 1u) ||
      ((uintptr_t)d_tsim_out & 1u) || ((uintptr_t)d_sigma_out & 3u))
    return fail_with(MPD_ERR_PTR, "state outputs NULL or misaligned");
  if (d_updates != nullptr && ((uintptr_t)d_updates & 7u)) return fail_with(MPD_ERR_PTR, "updates misaligned");
  AsyncArgs a = {};
  a.L = L;
  a.seeds = d_clock_seeds;
  a.links = d_links;
  a.ring_thr = ring_thr;
  a.t_target = t_target;
  a.S_max = S_max;
  a.sched = sched;
  a.slots = d_slots;
  a.updates = d_updates;
  a.syn = d_sigma_out;
  a.m_out = d_m_out;
  a.tsim_out = d_tsim_out;
  a.wind_out = d_wind_out;
  return launch_async(a, n, unc, (hipStream_t)stream);
}

extern "C" {

int mpd_decode_async(int L, double p, const uint64_t *d_seeds, int64_t n, double rho, int S_max, int32_t *d_T_async,
                     uint8_t *d_flags, int32_t *d_slots, int64_t *d_updates, uint32_t *d_final_syndrome,
                     void *stream) {
  g_last_error.clear();
  return decode_desync(false, 0, L, p, d_seeds, n, rho, S_max, d_T_async, d_flags, d_slots, d_updates, d_final_syndrome,
                       stream);
}

int mpd_run_async(int L, const uint32_t *d_links, const uint64_t *d_clock_seeds, int64_t n, int t_target, double rho,
                  int S_max, int32_t *d_slots, int64_t *d_updates, int16_t *d_m_out, uint16_t *d_tsim_out,
                  uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream) {
  g_last_error.clear();
  return run_desync(false, 0, L, d_links, d_clock_seeds, n, t_target, rho, S_max, d_slots, d_updates, d_m_out,
                    d_tsim_out, d_sigma_out, d_wind_out, stream);
}

int mpd_decode_uncoord(int L, double p, const uint64_t *d_seeds, int64_t n, double rho, int S_max, int schedule,
                       int32_t *d_T_un, uint8_t *d_flags, int32_t *d_slots, int64_t *d_updates,
                       uint32_t *d_final_syndrome, void *stream) {
  g_last_error.clear();
  if (schedule != MPD_UNCOORD_CYCLIC && schedule != MPD_UNCOORD_RANDOM)
    return fail_with(MPD_ERR_N, "unknown schedule %d", schedule);
  return decode_desync(true, schedule, L, p, d_seeds, n, rho, S_max, d_T_un, d_flags, d_slots, d_updates, d_final_syndrome,
                       stream);
}

int mpd_run_uncoord(int L, const uint32_t *d_links, const uint64_t *d_clock_seeds, int64_t n, int t_target,
                    double rho, int S_max, int schedule, int32_t *d_slots, int64_t *d_updates, int16_t *d_m_out,
                    uint16_t *d_tsim_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream) {
  g_last_error.clear();
  if (schedule != MPD_UNCOORD_CYCLIC && schedule != MPD_UNCOORD_RANDOM)
    return fail_with(MPD_ERR_N, "unknown schedule %d", schedule);
  return run_desync(true, schedule, L, d_links, d_clock_seeds, n, t_target, rho, S_max, d_slots, d_updates, d_m_out,
                    d_tsim_out, d_sigma_out, d_wind_out, stream);
}

}  // extern "C"
