/*
 * mpd_oracle.c -- CPU oracle for the synchronous 2D message-passing automaton
 * decoder of E. Lake, "Fast offline decoding with local message-passing
 * automata" (arXiv:2506.03266).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition that the
 * GPU path is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or helper with the HIP library and includes nothing from it.
 *
 * Everything here follows the paper's notation and order of operations:
 *   - qubits on the 2L^2 links of a periodic L x L square lattice, i.i.d. X
 *     noise of strength p on every link (Sec. 2.1, Sec. 2.2, Sec. 7);
 *   - syndrome sigma_r = -1 at a vertex touched by an odd number of flipped
 *     links (Def. "synchronous automaton decoder");
 *   - four message registers m^{+x}, m^{-x}, m^{+y}, m^{-y} per vertex,
 *     updated v times per decoder step by the rule A^{(D)} of
 *     Def. "message passing automaton, general dimensions" (Sec. 3.2), all
 *     sites simultaneously;
 *   - then one application of the feedback operators F^{(D)} of the same
 *     definition, with the degeneracy-breaking argmin' of eq. (degbreak) and
 *     the OR function of Def. "message passing automaton, 1D";
 *   - decoding time T_dec = number of decoder steps until no anyon is left
 *     (Def. "logical failure rate, expected decoding time, and thresholds");
 *   - logical failure = error + correction winds a non-trivial cycle of the
 *     torus (Sec. 7.2: either or both of the two cycles).
 *
 * Readings taken where the text is garbled or silent (each is listed with
 * its justification in the design notes of the repository):
 *   R1  C^{(a)}_r is the 3-site line through r normal to a.
 *   R2  the "min + 1" branch of A^{(D)} takes the minimum over NONZERO
 *       registers only (0 means "no message", Sec. 3.1).
 *   R3  in f^a = sgn(m^{-a} - m^{+a}) an absent message (0) counts as
 *       +infinity, i.e. an anyon moves toward the source of the smallest
 *       message it holds, and does not move on an exact tie along that axis.
 *   R4  only anyon sites (sigma = -1) apply feedback; f := 0 elsewhere.
 *   R5  argmin' compares the messages first and uses the offset s a/(D+1)
 *       only between equal messages (axis a = 1 is x, a = 2 is y), giving
 *       the order -y < -x < +x < +y on ties.  Read literally, m + s a/(D+1)
 *       would leave (-x, m+1) and (+y, m) tied, and (-y, m+1) tied with
 *       (+x, m), so it would not remove the degeneracies it is introduced to
 *       remove; the anyon is meant to follow its smallest message.
 *   R6  within one step the v message updates come first, then feedback;
 *       sigma is fixed during the message updates.
 *   R7  T_dec and T_max count decoder steps (feedback applications).
 *   R8  no truncation of message values (m_max = infinity).
 *   R9  periodic boundary conditions, L >= 3.
 *   R10 a sample still holding anyons after T_max steps is reported as a
 *       timeout, counted as a failure, with T_dec = T_max.
 *   R11 failure iff either winding parity of E + C is odd.
 *   R12 noise: Philox4x32-10 keyed by the 64-bit seed, counter = site-pair
 *       index; word 2(i&1) drives the x-link and word 2(i&1)+1 the y-link of
 *       site i; a link flips iff the word is below floor(p * 2^32).
 *
 * Limited classical memory (Sec. 5.3, the corollary on thresholds with
 * limited memory), an optional variant of the rule:
 *   R17 with a finite m_max, registers take values in {0, ..., m_max}: an
 *       update whose value would exceed m_max yields 0 (the message
 *       disappears).  m_max = 0 here means no truncation (R8).
 *   R18 with u > 0, at every decoder step t (counted from 1) with t a
 *       multiple of u, each anyon moves in a random direction instead of
 *       following its messages: Philox4x32-10 keyed by the sample's seed,
 *       counter (i >> 1, t, 0x4D4F5645, 0); word (i & 1) of site i, taken
 *       mod 4, gives +x, -x, +y, -y for 0..3.  Moves flip links through the
 *       same OR rule.  u = 0 means no random moves.
 *
 * Open boundaries (appendix "open boundaries", Def. "message passing
 * automaton with open boundaries"), an optional variant of the lattice:
 *   R19 sites (x, y), 0 <= x, y < L, no wrap; the rough boundary B is the
 *       columns x = 0 and x = L-1 (eq. (lrboundaries)); rows y = 0 and
 *       y = L-1 end without a boundary of that kind (smooth).
 *   R20 qubits are the links with a bulk endpoint: x-links (x,y)-(x+1,y)
 *       for x <= L-2, y-links (x,y)-(x,y+1) for y <= L-2 and 1 <= x <= L-2.
 *       Noise and explicit errors on other links are ignored.  Only bulk
 *       sites carry a syndrome; a string may end on B.
 *   R21 messages: registers at B sites are 0; m^{+x} (m^{-x}) is 1 at bulk
 *       sites whose left (right) neighbour is in B; lines are clipped to the
 *       lattice and empty when their centre lies outside it; otherwise the
 *       rule of R1-R2.  Feedback unchanged; an anyon moving onto B is
 *       absorbed.
 *   R22 one logical qubit: failure iff E + C crosses the cut between
 *       columns L-2 and L-1 an odd number of times (a string from B_L to
 *       B_R); timeouts count as failures.
 *
 * Marching-soldiers desynchronization (Sec. "Desynchronization and
 * Lindbladian dynamics"), an optional asynchronous driver of the plain rule
 * on the torus:
 *   R23 each decoder step is v + 1 automaton updates of a site: v message
 *       updates, then one feedback update that applies F to the two links
 *       the site owns (r -> r + x-hat, r -> r + y-hat).  The definition
 *       applies feedback together with the v-th update; its own update slot
 *       keeps v message updates per feedback and makes the simulated
 *       dynamics exactly F o A^v of R6.  t_sim counts these updates.
 *   R24 Delta = 1 (A and F read the 3 x 3 block around a site and F writes
 *       inside it); an update of r is accepted iff t_sim(q) >= t_sim(r) for
 *       every q != r with |q - r|_inf <= 2 Delta; a rejected one does nothing.
 *   R25 per-site state: m^old, m^new, the physical syndrome sigma and two
 *       flip parities acc[k mod 2] (flips applied at the site by the feedback
 *       of step k).  The present view of a neighbour q is m^new_q when level
 *       with r and m^old_q when one update ahead; a feedback update of step
 *       k reads sigma_q (-1)^{acc[k mod 2]_q}, a message update sigma_q as it
 *       is; a site's first update of step k clears its acc[(k-1) mod 2].  This
 *       stores what sigma^old, sigma^new and sigma^future store, with the
 *       reset tied to the site's own progress as in the definition.
 *   R26 clock: time runs in slots; in slot s site i rings iff word 2(i&1) of
 *       Philox4x32-10(key = seed, counter = (i >> 1, s, 0x41535943, 0)) is
 *       below ring_thr (a probability times 2^32), and ringing sites attempt
 *       one update each in increasing order of (top 19 bits of word
 *       2(i&1)+1, i), i.e. of word >> 13, then the site index.  As the
 *       probability goes to 0 with slots of that length this is the
 *       independent rate-1 Poisson clocks the section names as an example;
 *       the simulated decoder does not depend on the order (Prop. "faithful
 *       Lindbladian simulation").
 *   R27 a desynchronized decode ends at the first slot boundary where the
 *       physical syndrome holds no anyon and no acc bit is set: every view
 *       then holds no anyon, so no link can flip again.  T_async = 1 + the
 *       last slot with a flip (0 if none); outcome as R10, R11.
 *
 * Uncoordinated desynchronization (Sec. "Uncoordinated desynchronization"):
 *   R28 the same clock (R26) and update schedule (v message updates, then one
 *       motion update, cyclically), without the lag rule and without old
 *       copies: a message update reads the current registers and syndromes
 *       on its lines; a motion update of an anyon site moves that anyon one
 *       link along its force (+a for f^a = -1, -a for f^a = +1), which
 *       annihilates it with an anyon there.  A decode ends at the first slot
 *       boundary with no anyon; T_un = 1 + the last slot with a move.
 *       Schedule "cyclic": the (v+1)-th update of a site is a motion.
 *       Schedule "random": each update is a motion with probability
 *       1 / (v+1), independently: word (i & 1) of Philox4x32-10(key = seed,
 *       counter (i >> 1, slot, 0x54595045, 0)) mod (v+1) == v (the two kinds
 *       of updates then run on independent Poisson clocks of rates v and 1).
 *
 * Site index i = y*L + x.  The x-link of site (x,y) joins (x,y) and
 * (x+1,y); its y-link joins (x,y) and (x,y+1) (indices mod L).
 * Register order in every array: d = 0: +x, 1: -x, 2: +y, 3: -y, i.e.
 * (s,a) = (+1,1), (-1,1), (+1,2), (-1,2).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EBADARG -1
#define ORC_ENOMEM -2

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: the counter-based generator of Salmon, Moraes, Dror and    */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).  Ten rounds  */
/* of the multiply-hi/lo S-box with the Weyl-sequence key schedule.          */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k[2] = {key_in[0], key_in[1]};
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k[0] += W0;
      k[1] += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Flip threshold: a 32-bit uniform word u flips its link iff u < thr. */
static uint64_t orc_threshold(double p) {
  double t = floor(p * 4294967296.0);
  if (t < 0.0) t = 0.0;
  if (t > 4294967296.0) t = 4294967296.0;
  return (uint64_t)t;
}

/* i.i.d. bit-flip noise N on the 2L^2 links (R12).  ex/ey: L*L bytes. */
int orc_noise(int L, double p, uint64_t seed, uint8_t *ex, uint8_t *ey) {
  if (L < 3 || !(p >= 0.0 && p <= 1.0)) return ORC_EBADARG;
  uint64_t thr = orc_threshold(p);
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  int64_t nsite = (int64_t)L * L;
  for (int64_t i = 0; i < nsite; ++i) {
    uint32_t ctr[4] = {(uint32_t)(i >> 1), 0u, 0u, 0u};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    int half = (int)(i & 1);
    ex[i] = ((uint64_t)w[2 * half] < thr) ? 1 : 0;
    ey[i] = ((uint64_t)w[2 * half + 1] < thr) ? 1 : 0;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Decoder state                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
  int L, v;
  int open;           /* R19-R22: open boundaries instead of the torus */
  int m_max;          /* R17: 0 = no truncation */
  int u;              /* R18: 0 = no random moves */
  uint32_t key[2];    /* the sample's seed, for the random moves */
  int t;              /* the decoder step being applied (from 1) */
  int64_t n;          /* number of sites L*L */
  int32_t *m[4];      /* m^{sa}_r, registers after the last update */
  int32_t *mnew[4];   /* scratch for the synchronous update */
  int8_t *sigma;      /* +1 / -1 */
  uint8_t *cx, *cy;   /* correction chain C (links flipped by feedback) */
  int8_t *fx, *fy;    /* f^x_r, f^y_r of the current step */
  uint8_t *flx, *fly; /* link exponents of the current step */
} orc_state;

static const int DIR_S[4] = {+1, -1, +1, -1};
static const int DIR_A[4] = {1, 1, 2, 2};

/* Alternative readings of the garbled or ambiguous passages, for the
 * comparison with the paper's printed threshold and slope only (a script
 * beside this file tabulates them).  0, the default, is the reading R1-R5
 * above, which every decoder entry point and every test uses.  Bits:
 *   ORC_READ_LITERAL_SIGN  f^a = sgn(m^{-a} - m^{+a}) with an absent message
 *                          taken as the value 0 (instead of R3's +infinity)
 *   ORC_READ_LITERAL_KEY   argmin' minimises the number m + s a/(D+1) itself
 *                          (eq. (degbreak) as printed) instead of R5's
 *                          messages-first order
 *   ORC_READ_TIE_MOVES     an anyon whose two registers on the chosen axis
 *                          are equal still moves toward the source of the
 *                          chosen register (instead of sgn(0) = 0)
 *   ORC_READ_TIE_MIRROR    ties between equal messages in the order
 *                          +y < +x < -x < -y (R5 mirrored)
 *   ORC_READ_LINE_SITE     C^{(a)} is the single site r - s a-hat (the
 *                          1D rule applied per direction, no sideways spread)
 *   ORC_READ_LINE_BALL     C^{(a)} is the whole unit infinity-ball around
 *                          r - s a-hat (the printed constraint dropped)
 * Set once, before decoding; it is process-wide. */
#define ORC_READ_LITERAL_SIGN 1
#define ORC_READ_LITERAL_KEY 2
#define ORC_READ_TIE_MOVES 4
#define ORC_READ_TIE_MIRROR 8
#define ORC_READ_LINE_SITE 16
#define ORC_READ_LINE_BALL 32
#define ORC_READ_ALL 63
static int g_reading = 0;

int orc_set_reading(int r) {
  if (r < 0 || (r & ~ORC_READ_ALL) || ((r & ORC_READ_LINE_SITE) && (r & ORC_READ_LINE_BALL))) return ORC_EBADARG;
  g_reading = r;
  return ORC_OK;
}

int orc_get_reading(void) { return g_reading; }

static int wrap(int c, int L) {
  c %= L;
  return c < 0 ? c + L : c;
}

static void orc_free(orc_state *st) {
  for (int d = 0; d < 4; ++d) {
    free(st->m[d]);
    free(st->mnew[d]);
  }
  free(st->sigma); free(st->cx); free(st->cy);
  free(st->fx); free(st->fy); free(st->flx); free(st->fly);
  memset(st, 0, sizeof(*st));
}

static int orc_alloc(orc_state *st, int L, int v) {
  memset(st, 0, sizeof(*st));
  st->L = L; st->v = v; st->n = (int64_t)L * L;
  size_t n = (size_t)st->n;
  int ok = 1;
  for (int d = 0; d < 4; ++d) {
    st->m[d] = (int32_t *)calloc(n, sizeof(int32_t));
    st->mnew[d] = (int32_t *)calloc(n, sizeof(int32_t));
    ok = ok && st->m[d] && st->mnew[d];
  }
  st->sigma = (int8_t *)calloc(n, 1);
  st->cx = (uint8_t *)calloc(n, 1); st->cy = (uint8_t *)calloc(n, 1);
  st->fx = (int8_t *)calloc(n, 1); st->fy = (int8_t *)calloc(n, 1);
  st->flx = (uint8_t *)calloc(n, 1); st->fly = (uint8_t *)calloc(n, 1);
  ok = ok && st->sigma && st->cx && st->cy && st->fx && st->fy && st->flx && st->fly;
  if (!ok) { orc_free(st); return ORC_ENOMEM; }
  return ORC_OK;
}

/* Open boundaries: is column x part of the rough boundary B (R19)? */
static int orc_in_B(const orc_state *st, int x) { return st->open && (x == 0 || x == st->L - 1); }

/* Does the link of site (x, y) in direction dir (0: x-link, 1: y-link)
 * exist (R20)?  Every link does on the torus. */
static int orc_link_exists(const orc_state *st, int x, int y, int dir) {
  if (!st->open) return 1;
  if (dir == 0) return x <= st->L - 2;
  return y <= st->L - 2 && x >= 1 && x <= st->L - 2;
}

/* sigma = boundary of the error chain: -1 where an odd number of the four
 * incident links carry an error (Def. "synchronous automaton decoder").
 * With open boundaries only bulk sites carry a syndrome, and links that do
 * not exist must be 0 in ex / ey. */
static void orc_syndrome(orc_state *st, const uint8_t *ex, const uint8_t *ey) {
  int L = st->L;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int i = y * L + x;
      int par = ex[i] ^ ex[y * L + wrap(x - 1, L)] ^ ey[i] ^ ey[wrap(y - 1, L) * L + x];
      st->sigma[i] = (par && !orc_in_B(st, x)) ? -1 : +1;
    }
}

/* The value A^{(D)}, D = 2, gives register d of site (x, y) from the
 * registers m and syndrome sigma it reads.  For direction (s,a) the
 * register at r reads the line C^{(a)}_{r - s a}:
 *   1                                  if an anyon sits on the line,
 *   0                                  if every register on it is 0,
 *   (min of the nonzero registers) + 1 otherwise (R1, R2). */
static int32_t orc_register_value(const orc_state *st, int32_t *const m[4], const int8_t *sigma, int d, int x,
                                  int y) {
  int L = st->L;
  int s = DIR_S[d], a = DIR_A[d];
  int ax = (a == 1), ay = (a == 2);       /* unit vector a-hat */
  int bx = ay, by = ax;                   /* unit vector normal to a */
  int cxp = x - s * ax, cyp = y - s * ay; /* centre r - s a-hat */
  int anyon = 0;
  int32_t minnz = 0;
  if (st->open) {                                                    /* R21 */
    if (orc_in_B(st, x)) return 0;
    if (cxp < 0 || cxp >= L || cyp < 0 || cyp >= L) return 0;       /* empty line */
    if (orc_in_B(st, cxp)) anyon = 1;                                /* B sources x-messages */
  }
  /* the line C^{(a)}_{r - s a}: offsets k b-hat, |k| <= 1 (R1); the
   * alternative readings take the centre alone or the whole unit ball */
  int kmax = (g_reading & ORC_READ_LINE_SITE) ? 0 : 1;
  int jmax = (g_reading & ORC_READ_LINE_BALL) ? 1 : 0;
  for (int j = -jmax; j <= jmax; ++j)
  for (int k = -kmax; k <= kmax; ++k) {
    int qx = cxp + k * bx + j * ax, qy = cyp + k * by + j * ay;
    if (st->open && (qx < 0 || qx >= L || qy < 0 || qy >= L)) continue;   /* clipped */
    qx = wrap(qx, L);
    qy = wrap(qy, L);
    int q = qy * L + qx;
    if (sigma[q] == -1) anyon = 1;
    int32_t mv = m[d][q];
    if (mv > 0 && (minnz == 0 || mv < minnz)) minnz = mv;
  }
  int32_t out;
  if (anyon) out = 1;
  else if (minnz == 0) out = 0;
  else out = minnz + 1;
  if (st->m_max > 0 && out > st->m_max) out = 0;   /* R17 */
  return out;
}

/* One application of A^{(D)} to every register simultaneously. */
static void orc_message_update(orc_state *st) {
  int L = st->L;
  for (int d = 0; d < 4; ++d)
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) st->mnew[d][y * L + x] = orc_register_value(st, st->m, st->sigma, d, x, y);
  for (int d = 0; d < 4; ++d) {
    int32_t *t = st->m[d];
    st->m[d] = st->mnew[d];
    st->mnew[d] = t;
  }
}

/* sgn(mm - mp) with an absent message (0) read as +infinity (R3). */
static int orc_force(int32_t mp, int32_t mm) {
  if (g_reading & ORC_READ_LITERAL_SIGN) return (mm > mp) - (mm < mp);
  if (mp == 0 && mm == 0) return 0;
  if (mp == 0) return -1;   /* only m^{-a}: source on the +a side */
  if (mm == 0) return +1;   /* only m^{+a}: source on the -a side */
  return (mm > mp) - (mm < mp);
}

/* x OR y for x, y in {-1, 0, +1}: 1 iff either equals 1. */
static int orc_or(int x, int y) { return (x == 1 || y == 1) ? 1 : 0; }

/* Direction of the random move of site i at step t (R18): 0 +x, 1 -x,
 * 2 +y, 3 -y. */
static int orc_random_direction(const orc_state *st, int64_t i) {
  uint32_t ctr[4] = {(uint32_t)(i >> 1), (uint32_t)st->t, 0x4D4F5645u, 0u};
  uint32_t w[4];
  orc_philox4x32_10(ctr, st->key, w);
  return (int)(w[i & 1] & 3u);
}

/* The forces (f^x_r, f^y_r) of site i from the registers m and syndrome
 * sigma it reads, at decoder step st->t. */
static void orc_site_force(const orc_state *st, int32_t *const m[4], const int8_t *sigma, int64_t i, int8_t *fx,
                           int8_t *fy) {
  *fx = 0; *fy = 0;
  if (sigma[i] != -1) return;                   /* R4 */
  if (st->u > 0 && st->t % st->u == 0) {        /* R18 */
    /* The link exponent carries sigma_r f_r and sigma_r = -1 here, so an
     * anyon moves along +a for f^a = -1 (as for a force from orc_force). */
    int d = orc_random_direction(st, i);
    if (d < 2) *fx = (int8_t)(d == 0 ? -1 : +1);
    else *fy = (int8_t)(d == 2 ? -1 : +1);
    return;
  }
  int best = -1;
  int32_t bestm = 0, bestoff = 0;
  for (int d = 0; d < 4; ++d) {
    int32_t mv = m[d][i];
    if (mv <= 0) continue;
    /* argmin' of eq. (degbreak): the offset s a / (D+1) only breaks ties
     * between equal messages (R5): smallest m first, then smallest s*a. */
    int32_t off = DIR_S[d] * DIR_A[d];
    if (g_reading & ORC_READ_TIE_MIRROR) off = -off;
    int better;
    if (g_reading & ORC_READ_LITERAL_KEY)   /* m + s a/3 < m' + s' a'/3, in thirds */
      better = best < 0 || 3 * mv + off < 3 * bestm + bestoff;
    else
      better = best < 0 || mv < bestm || (mv == bestm && off < bestoff);
    if (better) {
      best = d;
      bestm = mv;
      bestoff = off;
    }
  }
  if (best < 0) return;                         /* M_r empty: no feedback */
  int f = DIR_A[best] == 1 ? orc_force(m[0][i], m[1][i]) : orc_force(m[2][i], m[3][i]);
  /* on an exact tie along the chosen axis: follow the chosen register
   * (source on the -s side, so the anyon moves along -s, i.e. f = s) */
  if (f == 0 && (g_reading & ORC_READ_TIE_MOVES)) f = DIR_S[best];
  if (DIR_A[best] == 1) *fx = (int8_t)f;
  else *fy = (int8_t)f;
}

/* The decision of a single site from its four registers (order +x, -x, +y,
 * -y) and its syndrome: the forces (f^x, f^y) of eq. (ddfeedback)'s
 * exponent, as the feedback of a plain-rule step computes them. */
int orc_decide(const int32_t m_in[4], int anyon, int *fx, int *fy) {
  orc_state st;
  memset(&st, 0, sizeof(st));
  st.L = 1;
  st.n = 1;
  int32_t reg[4];
  int32_t *m[4];
  for (int d = 0; d < 4; ++d) {
    if (m_in[d] < 0) return ORC_EBADARG;
    reg[d] = m_in[d];
    m[d] = &reg[d];
  }
  int8_t sigma = anyon ? -1 : +1, a = 0, b = 0;
  orc_site_force(&st, m, &sigma, 0, &a, &b);
  *fx = a;
  *fy = b;
  return ORC_OK;
}

/* Feedback F^{(D)}: per-site force f^a_r from argmin' over the nonzero
 * registers (ties broken by m + s a / (D+1), eq. (degbreak)), then the link
 * exponent sigma_r f^a_r OR sigma_{r+a}(-f^a_{r+a}) of eq. (ddfeedback).
 * Returns the number of anyons after the step. */
static int64_t orc_feedback(orc_state *st) {
  int L = st->L;
  int64_t n = st->n;
  for (int64_t i = 0; i < n; ++i) orc_site_force(st, st->m, st->sigma, i, &st->fx[i], &st->fy[i]);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int i = y * L + x;
      int ix = y * L + wrap(x + 1, L), iy = wrap(y + 1, L) * L + x;
      st->flx[i] = orc_link_exists(st, x, y, 0)
                       ? (uint8_t)orc_or(st->sigma[i] * st->fx[i], st->sigma[ix] * (-st->fx[ix])) : 0;
      st->fly[i] = orc_link_exists(st, x, y, 1)
                       ? (uint8_t)orc_or(st->sigma[i] * st->fy[i], st->sigma[iy] * (-st->fy[iy])) : 0;
    }
  int64_t anyons = 0;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int i = y * L + x;
      int par = st->flx[i] ^ st->flx[y * L + wrap(x - 1, L)] ^ st->fly[i] ^
                st->fly[wrap(y - 1, L) * L + x];
      st->cx[i] ^= st->flx[i];
      st->cy[i] ^= st->fly[i];
      if (par && !orc_in_B(st, x)) st->sigma[i] = (int8_t)(-st->sigma[i]);   /* B absorbs (R20) */
    }
  for (int64_t i = 0; i < n; ++i) anyons += (st->sigma[i] == -1);
  return anyons;
}

static int64_t orc_count_anyons(const orc_state *st) {
  int64_t a = 0;
  for (int64_t i = 0; i < st->n; ++i) a += (st->sigma[i] == -1);
  return a;
}

/* Winding parity of a chain across the fixed cuts: x-links leaving column
 * L-1 and y-links leaving row L-1 on the torus (R11); with open boundaries
 * the x-links from column L-2 to L-1 and no second cycle (R22). */
static void orc_winding(int L, int open, const uint8_t *cx, const uint8_t *cy, int *wx, int *wy) {
  int a = 0, b = 0;
  int cut = open ? L - 2 : L - 1;
  for (int y = 0; y < L; ++y) a ^= cx[y * L + cut];
  if (!open)
    for (int x = 0; x < L; ++x) b ^= cy[(L - 1) * L + x];
  *wx = a; *wy = b;
}

/* Copy of an error chain without the links that do not exist (R20). */
static int orc_masked_chain(const orc_state *st, const uint8_t *ex, const uint8_t *ey, uint8_t **mx,
                            uint8_t **my) {
  int L = st->L;
  *mx = (uint8_t *)malloc((size_t)st->n);
  *my = (uint8_t *)malloc((size_t)st->n);
  if (!*mx || !*my) { free(*mx); free(*my); return ORC_ENOMEM; }
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int i = y * L + x;
      (*mx)[i] = orc_link_exists(st, x, y, 0) ? ex[i] : 0;
      (*my)[i] = orc_link_exists(st, x, y, 1) ? ey[i] : 0;
    }
  return ORC_OK;
}

static void orc_pack_sigma(const orc_state *st, uint32_t *words) {
  int64_t nw = (st->n + 31) / 32;
  memset(words, 0, (size_t)nw * 4);
  for (int64_t i = 0; i < st->n; ++i)
    if (st->sigma[i] == -1) words[i >> 5] |= 1u << (i & 31);
}

/* ------------------------------------------------------------------------ */
/* Public entry points (used through ctypes by the tests)                    */
/* ------------------------------------------------------------------------ */

/* Decode one explicit error pattern.  Outputs T_dec, flags (bit0 = logical
 * failure, bit1 = timeout) and the final syndrome, packed as bit i%32 of
 * word i/32 for site i = y*L + x.  Optional outputs may be NULL:
 *   m_out     [4][L*L] int32 registers at the end,
 *   cx_out, cy_out  [L*L] correction chain,
 *   wind_out  [4] = (Wx_E, Wy_E, Wx_C, Wy_C). */
/* The same with the limited-memory variant: m_max (R17) and u (R18, random
 * moves keyed by `seed`). */
static int orc_decode_any(int L, int v, int open, int m_max, int u, uint64_t seed, const uint8_t *ex_in,
                          const uint8_t *ey_in, int T_max, int32_t *T_dec, uint8_t *flags,
                          uint32_t *sigma_words, int32_t *m_out, uint8_t *cx_out, uint8_t *cy_out,
                          int32_t *wind_out) {
  if (L < 3 || v < 1 || T_max < 0 || m_max < 0 || u < 0) return ORC_EBADARG;
  orc_state st;
  if (orc_alloc(&st, L, v) != ORC_OK) return ORC_ENOMEM;
  st.open = open;
  st.m_max = m_max;
  st.u = u;
  st.key[0] = (uint32_t)(seed & 0xffffffffu);
  st.key[1] = (uint32_t)(seed >> 32);
  uint8_t *ex, *ey;
  if (orc_masked_chain(&st, ex_in, ey_in, &ex, &ey) != ORC_OK) { orc_free(&st); return ORC_ENOMEM; }
  orc_syndrome(&st, ex, ey);
  int64_t anyons = orc_count_anyons(&st);
  int t = 0;
  while (anyons > 0 && t < T_max) {
    for (int j = 0; j < v; ++j) orc_message_update(&st);
    st.t = t + 1;
    anyons = orc_feedback(&st);
    ++t;
  }
  int wxe, wye, wxc, wyc;
  orc_winding(L, open, ex, ey, &wxe, &wye);
  orc_winding(L, open, st.cx, st.cy, &wxc, &wyc);
  free(ex);
  free(ey);
  int timeout = anyons > 0;
  int fail = timeout || ((wxe ^ wxc) | (wye ^ wyc));
  *T_dec = t;
  *flags = (uint8_t)((fail ? 1 : 0) | (timeout ? 2 : 0));
  if (sigma_words) orc_pack_sigma(&st, sigma_words);
  if (m_out)
    for (int d = 0; d < 4; ++d) memcpy(m_out + (size_t)d * st.n, st.m[d], (size_t)st.n * 4);
  if (cx_out) memcpy(cx_out, st.cx, (size_t)st.n);
  if (cy_out) memcpy(cy_out, st.cy, (size_t)st.n);
  if (wind_out) { wind_out[0] = wxe; wind_out[1] = wye; wind_out[2] = wxc; wind_out[3] = wyc; }
  orc_free(&st);
  return ORC_OK;
}

int orc_decode_errors_rule(int L, int v, int m_max, int u, uint64_t seed, const uint8_t *ex,
                           const uint8_t *ey, int T_max, int32_t *T_dec, uint8_t *flags,
                           uint32_t *sigma_words, int32_t *m_out, uint8_t *cx_out, uint8_t *cy_out,
                           int32_t *wind_out) {
  return orc_decode_any(L, v, 0, m_max, u, seed, ex, ey, T_max, T_dec, flags, sigma_words, m_out, cx_out,
                        cy_out, wind_out);
}

/* Open boundaries (R19-R22): wind_out[1] and [3] are 0. */
int orc_decode_errors_open(int L, int v, const uint8_t *ex, const uint8_t *ey, int T_max, int32_t *T_dec,
                           uint8_t *flags, uint32_t *sigma_words, int32_t *m_out, uint8_t *cx_out,
                           uint8_t *cy_out, int32_t *wind_out) {
  return orc_decode_any(L, v, 1, 0, 0, 0, ex, ey, T_max, T_dec, flags, sigma_words, m_out, cx_out, cy_out,
                        wind_out);
}

int orc_decode_errors(int L, int v, const uint8_t *ex, const uint8_t *ey, int T_max,
                      int32_t *T_dec, uint8_t *flags, uint32_t *sigma_words,
                      int32_t *m_out, uint8_t *cx_out, uint8_t *cy_out, int32_t *wind_out) {
  return orc_decode_errors_rule(L, v, 0, 0, 0, ex, ey, T_max, T_dec, flags, sigma_words, m_out, cx_out,
                                cy_out, wind_out);
}

/* Run exactly t_exact decoder steps (no early exit) from the noise pattern,
 * starting from m = 0.  Outputs the registers, the syndrome (+1/-1 bytes)
 * and the correction chain after the last step.  With record != NULL, the
 * anyon indicator after every step k = 0..t_exact is written to
 * record[k*L*L + i] (k = 0 is the initial syndrome). */
static int orc_run_any(int L, int v, int open, int m_max, int u, uint64_t seed, const uint8_t *ex_in,
                       const uint8_t *ey_in, int t_exact, int32_t *m_out, int8_t *sigma_out, uint8_t *cx_out,
                       uint8_t *cy_out, uint8_t *record) {
  if (L < 3 || v < 1 || t_exact < 0 || m_max < 0 || u < 0) return ORC_EBADARG;
  orc_state st;
  if (orc_alloc(&st, L, v) != ORC_OK) return ORC_ENOMEM;
  st.open = open;
  st.m_max = m_max;
  st.u = u;
  st.key[0] = (uint32_t)(seed & 0xffffffffu);
  st.key[1] = (uint32_t)(seed >> 32);
  uint8_t *ex, *ey;
  if (orc_masked_chain(&st, ex_in, ey_in, &ex, &ey) != ORC_OK) { orc_free(&st); return ORC_ENOMEM; }
  orc_syndrome(&st, ex, ey);
  free(ex);
  free(ey);
  if (record)
    for (int64_t i = 0; i < st.n; ++i) record[i] = st.sigma[i] == -1;
  for (int t = 0; t < t_exact; ++t) {
    for (int j = 0; j < v; ++j) orc_message_update(&st);
    st.t = t + 1;
    orc_feedback(&st);
    if (record)
      for (int64_t i = 0; i < st.n; ++i)
        record[(size_t)(t + 1) * st.n + i] = st.sigma[i] == -1;
  }
  if (m_out)
    for (int d = 0; d < 4; ++d) memcpy(m_out + (size_t)d * st.n, st.m[d], (size_t)st.n * 4);
  if (sigma_out) memcpy(sigma_out, st.sigma, (size_t)st.n);
  if (cx_out) memcpy(cx_out, st.cx, (size_t)st.n);
  if (cy_out) memcpy(cy_out, st.cy, (size_t)st.n);
  orc_free(&st);
  return ORC_OK;
}

int orc_run_steps_rule(int L, int v, int m_max, int u, uint64_t seed, const uint8_t *ex,
                       const uint8_t *ey, int t_exact, int32_t *m_out, int8_t *sigma_out, uint8_t *cx_out,
                       uint8_t *cy_out, uint8_t *record) {
  return orc_run_any(L, v, 0, m_max, u, seed, ex, ey, t_exact, m_out, sigma_out, cx_out, cy_out, record);
}

int orc_run_steps_open(int L, int v, const uint8_t *ex, const uint8_t *ey, int t_exact, int32_t *m_out,
                       int8_t *sigma_out, uint8_t *cx_out, uint8_t *cy_out, uint8_t *record) {
  return orc_run_any(L, v, 1, 0, 0, 0, ex, ey, t_exact, m_out, sigma_out, cx_out, cy_out, record);
}

int orc_run_steps(int L, int v, const uint8_t *ex, const uint8_t *ey, int t_exact,
                  int32_t *m_out, int8_t *sigma_out, uint8_t *cx_out, uint8_t *cy_out,
                  uint8_t *record) {
  return orc_run_steps_rule(L, v, 0, 0, 0, ex, ey, t_exact, m_out, sigma_out, cx_out, cy_out, record);
}

/* Noise + decode for a batch of seeds; samples are spread over nthreads
 * OpenMP threads (nthreads <= 0: the OpenMP default).  Returns the number
 * of threads actually used through *threads_used. */
static int orc_seeds_any(int L, int v, int open, int m_max, int u, const double *p, int p_stride,
                         const uint64_t *seeds, int64_t n, int T_max, int nthreads, int32_t *T_dec,
                         uint8_t *flags, uint32_t *sigma_words, int *threads_used) {
  if (L < 3 || v < 1 || T_max < 0 || n < 0 || m_max < 0 || u < 0) return ORC_EBADARG;
  int64_t nsite = (int64_t)L * L;
  int64_t nw = (nsite + 31) / 32;
  int err = ORC_OK;
  int used = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
#else
  (void)nthreads;
#endif
  if (threads_used) *threads_used = used;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n; ++k) {
    uint8_t *ex = (uint8_t *)malloc((size_t)nsite);
    uint8_t *ey = (uint8_t *)malloc((size_t)nsite);
    int rc = (ex && ey) ? ORC_OK : ORC_ENOMEM;
    if (rc == ORC_OK) rc = orc_noise(L, p[p_stride ? k : 0], seeds[k], ex, ey);
    if (rc == ORC_OK)
      rc = orc_decode_any(L, v, open, m_max, u, seeds[k], ex, ey, T_max, &T_dec[k], &flags[k],
                          sigma_words ? sigma_words + k * nw : NULL, NULL, NULL, NULL, NULL);
    if (rc != ORC_OK) {
#pragma omp critical
      err = rc;
    }
    free(ex);
    free(ey);
  }
  return err;
}

int orc_decode_seeds_rule(int L, int v, int m_max, int u, const double *p, int p_stride,
                          const uint64_t *seeds, int64_t n, int T_max, int nthreads, int32_t *T_dec,
                          uint8_t *flags, uint32_t *sigma_words, int *threads_used) {
  return orc_seeds_any(L, v, 0, m_max, u, p, p_stride, seeds, n, T_max, nthreads, T_dec, flags, sigma_words,
                       threads_used);
}

int orc_decode_seeds_open(int L, int v, const double *p, int p_stride, const uint64_t *seeds, int64_t n,
                          int T_max, int nthreads, int32_t *T_dec, uint8_t *flags, uint32_t *sigma_words,
                          int *threads_used) {
  return orc_seeds_any(L, v, 1, 0, 0, p, p_stride, seeds, n, T_max, nthreads, T_dec, flags, sigma_words,
                       threads_used);
}

int orc_decode_seeds(int L, int v, const double *p, int p_stride, const uint64_t *seeds,
                     int64_t n, int T_max, int nthreads, int32_t *T_dec, uint8_t *flags,
                     uint32_t *sigma_words, int *threads_used) {
  return orc_seeds_any(L, v, 0, 0, 0, p, p_stride, seeds, n, T_max, nthreads, T_dec, flags, sigma_words,
                       threads_used);
}

/* Decode a batch of explicit error chains given as link bits: link id
 * l = 2*i + dir (dir 0: x-link of site i, dir 1: y-link), bit l%32 of word
 * l/32, ceil(2*L*L/32) words per sample. */
static int orc_links_any(int L, int v, int open, int m_max, int u, const uint64_t *seeds, const uint32_t *links,
                         int64_t n, int T_max, int nthreads, int32_t *T_dec, uint8_t *flags,
                         uint32_t *sigma_words) {
  if (L < 3 || v < 1 || T_max < 0 || n < 0 || m_max < 0 || u < 0) return ORC_EBADARG;
  if (u > 0 && seeds == NULL) return ORC_EBADARG;
  int64_t nsite = (int64_t)L * L;
  int64_t lw = (2 * nsite + 31) / 32, nw = (nsite + 31) / 32;
  int err = ORC_OK;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < n; ++k) {
    uint8_t *ex = (uint8_t *)malloc((size_t)nsite);
    uint8_t *ey = (uint8_t *)malloc((size_t)nsite);
    int rc = (ex && ey) ? ORC_OK : ORC_ENOMEM;
    if (rc == ORC_OK) {
      const uint32_t *w = links + k * lw;
      for (int64_t i = 0; i < nsite; ++i) {
        int64_t lx = 2 * i, ly = 2 * i + 1;
        ex[i] = (uint8_t)((w[lx >> 5] >> (lx & 31)) & 1u);
        ey[i] = (uint8_t)((w[ly >> 5] >> (ly & 31)) & 1u);
      }
      rc = orc_decode_any(L, v, open, m_max, u, seeds ? seeds[k] : 0, ex, ey, T_max, &T_dec[k], &flags[k],
                          sigma_words ? sigma_words + k * nw : NULL, NULL, NULL, NULL, NULL);
    }
    if (rc != ORC_OK) {
#pragma omp critical
      err = rc;
    }
    free(ex);
    free(ey);
  }
  return err;
}

int orc_decode_links_rule(int L, int v, int m_max, int u, const uint64_t *seeds, const uint32_t *links,
                          int64_t n, int T_max, int nthreads, int32_t *T_dec, uint8_t *flags,
                          uint32_t *sigma_words) {
  return orc_links_any(L, v, 0, m_max, u, seeds, links, n, T_max, nthreads, T_dec, flags, sigma_words);
}

int orc_decode_links_open(int L, int v, const uint32_t *links, int64_t n, int T_max, int nthreads,
                          int32_t *T_dec, uint8_t *flags, uint32_t *sigma_words) {
  return orc_links_any(L, v, 1, 0, 0, NULL, links, n, T_max, nthreads, T_dec, flags, sigma_words);
}

int orc_decode_links(int L, int v, const uint32_t *links, int64_t n, int T_max, int nthreads,
                     int32_t *T_dec, uint8_t *flags, uint32_t *sigma_words) {
  return orc_links_any(L, v, 0, 0, 0, NULL, links, n, T_max, nthreads, T_dec, flags, sigma_words);
}

/* ------------------------------------------------------------------------ */
/* Desynchronized decoders, torus only: marching soldiers (Sec.             */
/* "Desynchronization and Lindbladian dynamics": Def. "simulation and lag   */
/* times", Def. "marching soldiers desynchronization", Def. "desynchronized */
/* decoders", Prop. "faithful Lindbladian simulation"; readings R23-R27)    */
/* and the uncoordinated desynchronization (Sec. "Uncoordinated             */
/* desynchronization"; reading R28), on one clock.                          */
/* ------------------------------------------------------------------------ */
#define ORC_CLOCK_TAG 0x41535943u
#define ORC_TYPE_TAG 0x54595045u
#define ORC_EBROKEN -3   /* a lag left {0, 1} inside the update ball */

typedef struct {
  orc_state st;        /* st.m = m^new, st.sigma = the physical syndrome, st.cx / st.cy = C */
  int32_t *mold[4];    /* m^old */
  int32_t *pm[4];      /* the present view (m^present) around the updating site */
  int8_t *ps;          /* sigma^present around the updating site */
  int32_t *tsim;       /* t_sim: updates performed at each site */
  uint8_t *acc[2];     /* flips applied at each site by the feedback of step k, slot k mod 2 (R25) */
  int64_t updates;     /* accepted updates */
  int64_t flips;       /* links flipped */
  int unc;             /* uncoordinated desynchronization (R28) instead of marching soldiers */
  int sched;           /* R28 schedule: 0 cyclic, 1 random update types */
  int32_t slot;        /* the slot being run */
} orc_async;

static void orc_async_free(orc_async *a) {
  for (int d = 0; d < 4; ++d) { free(a->mold[d]); free(a->pm[d]); }
  free(a->ps); free(a->tsim); free(a->acc[0]); free(a->acc[1]);
  orc_free(&a->st);
}

static int orc_async_alloc(orc_async *a, int L, int v) {
  memset(a, 0, sizeof(*a));
  if (orc_alloc(&a->st, L, v) != ORC_OK) return ORC_ENOMEM;
  size_t n = (size_t)a->st.n;
  int ok = 1;
  for (int d = 0; d < 4; ++d) {
    a->mold[d] = (int32_t *)calloc(n, 4);
    a->pm[d] = (int32_t *)calloc(n, 4);
    ok = ok && a->mold[d] && a->pm[d];
  }
  a->ps = (int8_t *)calloc(n, 1);
  a->tsim = (int32_t *)calloc(n, 4);
  a->acc[0] = (uint8_t *)calloc(n, 1);
  a->acc[1] = (uint8_t *)calloc(n, 1);
  ok = ok && a->ps && a->tsim && a->acc[0] && a->acc[1];
  if (!ok) { orc_async_free(a); return ORC_ENOMEM; }
  return ORC_OK;
}

/* One update of site (x, y) of the uncoordinated desynchronization (R28):
 * no lag rule, current values only.  Returns 1 (every update is applied). */
static int orc_uncoord_update(orc_async *a, int x, int y) {
  orc_state *st = &a->st;
  int L = st->L, v = st->v;
  int64_t r = (int64_t)y * L + x;
  int32_t j = a->tsim[r];
  int motion;
  if (a->sched == 0) {
    motion = j % (v + 1) == v;
  } else {
    uint32_t ctr[4] = {(uint32_t)(r >> 1), (uint32_t)a->slot, ORC_TYPE_TAG, 0u}, w[4];
    orc_philox4x32_10(ctr, st->key, w);
    motion = w[r & 1] % (uint32_t)(v + 1) == (uint32_t)v;
  }
  if (!motion) {
    int32_t out[4];
    for (int d = 0; d < 4; ++d) out[d] = orc_register_value(st, st->m, st->sigma, d, x, y);
    for (int d = 0; d < 4; ++d) st->m[d][r] = out[d];
  } else if (st->sigma[r] == -1) {
    /* the anyon at r moves one link along its force: +a for f^a = -1, -a for
     * f^a = +1 (the sign of the link exponent sigma_r f_r with sigma_r = -1) */
    int8_t fx, fy;
    st->t = j / (v + 1) + 1;
    orc_site_force(st, st->m, st->sigma, r, &fx, &fy);
    int64_t q = -1;
    if (fx == -1) { st->cx[r] ^= 1; q = (int64_t)y * L + wrap(x + 1, L); }
    else if (fx == 1) { q = (int64_t)y * L + wrap(x - 1, L); st->cx[q] ^= 1; }
    else if (fy == -1) { st->cy[r] ^= 1; q = (int64_t)wrap(y + 1, L) * L + x; }
    else if (fy == 1) { q = (int64_t)wrap(y - 1, L) * L + x; st->cy[q] ^= 1; }
    if (q >= 0) {
      st->sigma[r] = (int8_t)(-st->sigma[r]);
      st->sigma[q] = (int8_t)(-st->sigma[q]);
      ++a->flips;
    }
  }
  a->tsim[r] = j + 1;
  ++a->updates;
  return 1;
}

/* One attempted automaton update of site (x, y) of the desynchronized
 * decoder.  Returns 1 if accepted, 0 if rejected, ORC_EBROKEN if the present
 * view could not be formed (a neighbour neither level with nor one update
 * ahead of the site, which the acceptance rule excludes). */
static int orc_async_update(orc_async *a, int x, int y) {
  orc_state *st = &a->st;
  int L = st->L, v = st->v;
  int64_t r = (int64_t)y * L + x;
  int32_t j = a->tsim[r];
  /* R24: accepted only if no site of the ball of radius 2 Delta is behind. */
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx) {
      if (!dx && !dy) continue;
      if (a->tsim[wrap(y + dy, L) * L + wrap(x + dx, L)] < j) return 0;
    }
  int k = j / (v + 1), phase = j % (v + 1);
  int feedback = phase == v;                    /* R23 */
  /* The present view of the ball of radius Delta (R25): a level neighbour
   * shows m^new, a neighbour one update ahead m^old; during a feedback
   * update sigma excludes the flips of this step already applied. */
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      int64_t q = (int64_t)wrap(y + dy, L) * L + wrap(x + dx, L);
      int32_t lag = a->tsim[q] - j;
      if (lag != 0 && lag != 1) return ORC_EBROKEN;
      for (int d = 0; d < 4; ++d) a->pm[d][q] = lag == 0 ? st->m[d][q] : a->mold[d][q];
      a->ps[q] = feedback && a->acc[k & 1][q] ? (int8_t)(-st->sigma[q]) : st->sigma[q];
    }
  if (!feedback) {
    if (phase == 0 && k > 0) a->acc[(k - 1) & 1][r] = 0;   /* R25: last step's flips are seen by all */
    int32_t out[4];
    for (int d = 0; d < 4; ++d) out[d] = orc_register_value(st, a->pm, a->ps, d, x, y);
    for (int d = 0; d < 4; ++d) {
      a->mold[d][r] = st->m[d][r];
      st->m[d][r] = out[d];
    }
  } else {
    /* F of the links r -> r + x-hat and r -> r + y-hat, from the present
     * view, as in orc_feedback. */
    st->t = k + 1;
    int64_t rx = (int64_t)y * L + wrap(x + 1, L), ry = (int64_t)wrap(y + 1, L) * L + x;
    int8_t fxr, fyr, fxx, fyx, fxy, fyy;
    orc_site_force(st, a->pm, a->ps, r, &fxr, &fyr);
    orc_site_force(st, a->pm, a->ps, rx, &fxx, &fyx);
    orc_site_force(st, a->pm, a->ps, ry, &fxy, &fyy);
    int lx = orc_or(a->ps[r] * fxr, a->ps[rx] * (-fxx));
    int ly = orc_or(a->ps[r] * fyr, a->ps[ry] * (-fyy));
    uint8_t *acc = a->acc[k & 1];
    if (lx) {
      st->cx[r] ^= 1;
      st->sigma[r] = (int8_t)(-st->sigma[r]); st->sigma[rx] = (int8_t)(-st->sigma[rx]);
      acc[r] ^= 1; acc[rx] ^= 1;
      ++a->flips;
    }
    if (ly) {
      st->cy[r] ^= 1;
      st->sigma[r] = (int8_t)(-st->sigma[r]); st->sigma[ry] = (int8_t)(-st->sigma[ry]);
      acc[r] ^= 1; acc[ry] ^= 1;
      ++a->flips;
    }
    for (int d = 0; d < 4; ++d) a->mold[d][r] = st->m[d][r];
  }
  a->tsim[r] = j + 1;
  ++a->updates;
  return 1;
}

typedef struct { uint32_t prio; int32_t i; } orc_ring;

static int orc_ring_cmp(const void *pa, const void *pb) {
  const orc_ring *a = (const orc_ring *)pa, *b = (const orc_ring *)pb;
  if (a->prio != b->prio) return a->prio < b->prio ? -1 : 1;
  return (a->i > b->i) - (a->i < b->i);
}

/* The desynchronized decoder on one error chain (torus, L >= 5).
 *   t_target >= 0: run until every site has performed (v+1) t_target
 *       updates (sites that have stop attempting), or S_max slots;
 *       flags bit1 set if the target was not reached.
 *   t_target < 0: decode -- run until the physical syndrome holds no anyon
 *       and no flip of any step is pending (R27), or S_max slots (timeout,
 *       flags bit1); flags bit0 = logical failure or timeout (R10, R11).
 * The clock (R26) is keyed by `seed`; ring_thr in [1, 2^32] is the ring
 * probability per slot times 2^32.  Outputs: slots run, T_async = 1 + the
 * slot of the last flip (0 if none), accepted updates, and optionally the
 * final syndrome words, m^new [4][L*L], t_sim [L*L] and the chain C. */
static int orc_desync_run(int unc, int sched, int L, int v, uint64_t seed, uint64_t ring_thr, const uint8_t *ex,
                          const uint8_t *ey, int t_target, int S_max, int32_t *slots_out, int32_t *T_async,
                          uint8_t *flags, int64_t *updates_out, uint32_t *sigma_words, int32_t *m_out,
                          int32_t *tsim_out, uint8_t *cx_out, uint8_t *cy_out) {
  if (L < 5 || v < 1 || S_max < 0 || ring_thr < 1 || ring_thr > ((uint64_t)1 << 32)) return ORC_EBADARG;
  orc_async a;
  if (orc_async_alloc(&a, L, v) != ORC_OK) return ORC_ENOMEM;
  a.unc = unc;
  a.sched = sched;
  orc_state *st = &a.st;
  st->key[0] = (uint32_t)(seed & 0xffffffffu);
  st->key[1] = (uint32_t)(seed >> 32);
  orc_syndrome(st, ex, ey);
  int64_t n = st->n;
  int32_t target = t_target >= 0 ? (v + 1) * t_target : 0;
  orc_ring *ring = (orc_ring *)malloc((size_t)n * sizeof(orc_ring));
  if (!ring) { orc_async_free(&a); return ORC_ENOMEM; }
  int rc = ORC_OK, done = 0;
  int32_t slot = 0, last_flip = -1;
  for (;;) {
    /* stop test at the start of each slot (before the first: nothing to do) */
    if (t_target >= 0) {
      done = 1;
      for (int64_t i = 0; i < n; ++i) done = done && a.tsim[i] >= target;
    } else {
      done = 1;
      for (int64_t i = 0; i < n; ++i) done = done && st->sigma[i] == 1 && !a.acc[0][i] && !a.acc[1][i];
    }
    if (done || slot >= S_max) break;
    /* R26: who rings in this slot, and in which order */
    int64_t nr = 0;
    for (int64_t i = 0; i < n; i += 2) {
      uint32_t ctr[4] = {(uint32_t)(i >> 1), (uint32_t)slot, ORC_CLOCK_TAG, 0u}, w[4];
      orc_philox4x32_10(ctr, st->key, w);
      for (int h = 0; h < 2 && i + h < n; ++h)
        if ((uint64_t)w[2 * h] < ring_thr) { ring[nr].prio = w[2 * h + 1] >> 13; ring[nr].i = (int32_t)(i + h); ++nr; }
    }
    qsort(ring, (size_t)nr, sizeof(orc_ring), orc_ring_cmp);
    int64_t f0 = a.flips;
    a.slot = slot;
    for (int64_t q = 0; q < nr && rc == ORC_OK; ++q) {
      int32_t i = ring[q].i;
      if (t_target >= 0 && a.tsim[i] >= target) continue;
      int got = a.unc ? orc_uncoord_update(&a, i % L, i / L) : orc_async_update(&a, i % L, i / L);
      if (got < 0) rc = got;
    }
    if (rc != ORC_OK) break;
    if (a.flips != f0) last_flip = slot;
    ++slot;
  }
  free(ring);
  if (rc == ORC_OK) {
    int wxe, wye, wxc, wyc;
    orc_winding(L, 0, ex, ey, &wxe, &wye);
    orc_winding(L, 0, st->cx, st->cy, &wxc, &wyc);
    int timeout = !done;
    int fail = t_target < 0 && (timeout || ((wxe ^ wxc) | (wye ^ wyc)));
    if (slots_out) *slots_out = slot;
    if (T_async) *T_async = last_flip + 1;
    if (flags) *flags = (uint8_t)((fail ? 1 : 0) | (timeout ? 2 : 0));
    if (updates_out) *updates_out = a.updates;
    if (sigma_words) orc_pack_sigma(st, sigma_words);
    if (m_out)
      for (int d = 0; d < 4; ++d) memcpy(m_out + (size_t)d * n, st->m[d], (size_t)n * 4);
    if (tsim_out) memcpy(tsim_out, a.tsim, (size_t)n * 4);
    if (cx_out) memcpy(cx_out, st->cx, (size_t)n);
    if (cy_out) memcpy(cy_out, st->cy, (size_t)n);
  }
  orc_async_free(&a);
  return rc;
}

int orc_async_run(int L, int v, uint64_t seed, uint64_t ring_thr, const uint8_t *ex, const uint8_t *ey,
                  int t_target, int S_max, int32_t *slots_out, int32_t *T_async, uint8_t *flags,
                  int64_t *updates_out, uint32_t *sigma_words, int32_t *m_out, int32_t *tsim_out,
                  uint8_t *cx_out, uint8_t *cy_out) {
  return orc_desync_run(0, 0, L, v, seed, ring_thr, ex, ey, t_target, S_max, slots_out, T_async, flags, updates_out,
                        sigma_words, m_out, tsim_out, cx_out, cy_out);
}

/* The uncoordinated desynchronization (R28) with the same clock, outputs
 * and stopping rules; t_sim counts every update; sched 0 cyclic, 1 random
 * update types. */
int orc_uncoord_run(int L, int v, int sched, uint64_t seed, uint64_t ring_thr, const uint8_t *ex, const uint8_t *ey,
                    int t_target, int S_max, int32_t *slots_out, int32_t *T_un, uint8_t *flags,
                    int64_t *updates_out, uint32_t *sigma_words, int32_t *m_out, int32_t *tsim_out,
                    uint8_t *cx_out, uint8_t *cy_out) {
  if (sched < 0 || sched > 1) return ORC_EBADARG;
  return orc_desync_run(1, sched, L, v, seed, ring_thr, ex, ey, t_target, S_max, slots_out, T_un, flags, updates_out,
                        sigma_words, m_out, tsim_out, cx_out, cy_out);
}

/* Noise (R12) + desynchronized decode for a batch of seeds, spread over
 * OpenMP threads; the seed keys both the noise and the clock. */
static int orc_desync_seeds(int unc, int sched, int L, int v, const double *p, int p_stride, const uint64_t *seeds, int64_t n,
                            uint64_t ring_thr, int S_max, int nthreads, int32_t *T_async, uint8_t *flags,
                            int32_t *slots_out, int64_t *updates_out, uint32_t *sigma_words, int *threads_used) {
  if (L < 5 || v < 1 || n < 0 || S_max < 0) return ORC_EBADARG;
  int64_t nsite = (int64_t)L * L, nw = (nsite + 31) / 32;
  int err = ORC_OK, used = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
#else
  (void)nthreads;
#endif
  if (threads_used) *threads_used = used;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n; ++k) {
    uint8_t *ex = (uint8_t *)malloc((size_t)nsite);
    uint8_t *ey = (uint8_t *)malloc((size_t)nsite);
    int rc = (ex && ey) ? ORC_OK : ORC_ENOMEM;
    if (rc == ORC_OK) rc = orc_noise(L, p[p_stride ? k : 0], seeds[k], ex, ey);
    if (rc == ORC_OK)
      rc = orc_desync_run(unc, sched, L, v, seeds[k], ring_thr, ex, ey, -1, S_max, &slots_out[k], &T_async[k], &flags[k],
                          &updates_out[k], sigma_words ? sigma_words + k * nw : NULL, NULL, NULL, NULL, NULL);
    if (rc != ORC_OK) {
#pragma omp critical
      err = rc;
    }
    free(ex);
    free(ey);
  }
  return err;
}

int orc_async_decode_seeds(int L, int v, const double *p, int p_stride, const uint64_t *seeds, int64_t n,
                           uint64_t ring_thr, int S_max, int nthreads, int32_t *T_async, uint8_t *flags,
                           int32_t *slots_out, int64_t *updates_out, uint32_t *sigma_words, int *threads_used) {
  return orc_desync_seeds(0, 0, L, v, p, p_stride, seeds, n, ring_thr, S_max, nthreads, T_async, flags, slots_out,
                          updates_out, sigma_words, threads_used);
}

int orc_uncoord_decode_seeds(int L, int v, int sched, const double *p, int p_stride, const uint64_t *seeds,
                             int64_t n, uint64_t ring_thr, int S_max, int nthreads, int32_t *T_un, uint8_t *flags,
                             int32_t *slots_out, int64_t *updates_out, uint32_t *sigma_words, int *threads_used) {
  if (sched < 0 || sched > 1) return ORC_EBADARG;
  return orc_desync_seeds(1, sched, L, v, p, p_stride, seeds, n, ring_thr, S_max, nthreads, T_un, flags, slots_out,
                          updates_out, sigma_words, threads_used);
}
