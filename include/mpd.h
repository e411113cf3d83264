/*
 * mpd.h -- C ABI of the MI355X message-passing decoder for the 2D toric code.
 *
 * The decoder is the synchronous automaton decoder of E. Lake, "Fast offline
 * decoding with local message-passing automata" (arXiv:2506.03266):
 *   - noise: i.i.d. bit flips of strength p on the 2L^2 links of an L x L
 *     periodic lattice (Sec. 2.2, eq. (final_channel); numerics of Sec. 7);
 *   - syndrome sigma measured once, then per decoder step v = 3 applications
 *     of the message rule A^{(D)} followed by one application of the feedback
 *     operators F^{(D)} (Def. "synchronous automaton decoder", Sec. 2.1;
 *     Def. "message passing automaton, general dimensions", Sec. 3.2);
 *   - stop at the first step with no anyon: T_dec (Def. "logical failure
 *     rate, expected decoding time, and thresholds", Sec. 5.1);
 *   - logical failure iff error + correction winds either cycle of the torus
 *     (Sec. 7.2).
 *
 * Conventions shared by every entry point
 *   - Site index i = y*L + x, 0 <= x, y < L.  The x-link of site (x,y) joins
 *     (x,y)-(x+1,y), its y-link joins (x,y)-(x,y+1), indices mod L.
 *   - Noise (seeded entry points): for site i, Philox4x32-10 (Salmon et al.,
 *     SC'11) with key = (seed & 0xffffffff, seed >> 32) and counter
 *     (i >> 1, 0, 0, 0); word 2*(i&1) drives the x-link and word 2*(i&1)+1 the
 *     y-link; a link flips iff word < floor(p * 2^32) (computed in double).
 *   - Link bit arrays: link id l = 2*i + dir (dir 0: x-link, 1: y-link), bit
 *     l % 32 of word l / 32, ceil(2*L*L/32) words per sample.
 *   - Syndrome bit arrays: bit i % 32 of word i / 32 set iff site i holds an
 *     anyon, ceil(L*L/32) words per sample.
 *   - flags: bit 0 (MPD_FLAG_FAIL) logical failure, bit 1 (MPD_FLAG_TIMEOUT)
 *     anyons left after T_max steps (then T_dec = T_max and the failure bit is
 *     also set).
 *   - Readings of the paper where it is silent or garbled: the message rule
 *     takes the minimum over nonzero registers only; an anyon moves toward the
 *     source of its smallest message, ties broken in the order
 *     -y < -x < +x < +y, and does not move on an exact tie along the chosen
 *     axis; only anyon sites apply feedback; messages are never truncated.
 *
 * Ownership and execution
 *   - Every pointer named d_* is caller-owned device memory on the current
 *     HIP device; the library never allocates, frees or keeps it.  Host
 *     memory is never read or written except the scalar arguments.  The
 *     library keeps, per host thread and device, a few streams and events of
 *     its own, and per host thread a small pinned host block for the pass
 *     counters (created on first use, kept until the process ends).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default
 *     stream).  Outputs are valid once the stream has reached the point after
 *     the call.  Calls that share a workspace must be ordered on one stream.
 *     Calls on different streams with separate workspaces may run
 *     concurrently from several host threads; their kernels then overlap on
 *     the device (one batch's short final passes fill in around another's).
 *   - Lattices up to L = 128 decode in a single launch with no host
 *     synchronization.  The large-lattice (band) path runs its later passes
 *     either from the host, reading a survivor counter back before each pass
 *     (the call then synchronizes `stream`), or on the device with no host
 *     wait (see mpd_set_band_driver).  A call on a stream that is being
 *     captured into a HIP graph always takes the device, so every
 *     mpd_decode_batch and mpd_decode_learned can be captured.
 *   - Return value 0 on success, a negative MPD_ERR_* code otherwise; the
 *     message of the last failing call on this host thread is returned by
 *     mpd_last_error().  On an error nothing has been enqueued unless the
 *     code is MPD_ERR_HIP.
 */
#ifndef MPD_H
#define MPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPD_OK 0
#define MPD_ERR_L (-1)         /* L unsupported for the call */
#define MPD_ERR_P (-2)         /* p is NaN or outside [0, 1] */
#define MPD_ERR_TMAX (-3)      /* T_max (or t_exact) outside [0, MPD_T_MAX_LIMIT] */
#define MPD_ERR_PTR (-4)       /* a required pointer is NULL or misaligned */
#define MPD_ERR_WORKSPACE (-5) /* ws_bytes < mpd_workspace_bytes(...) */
#define MPD_ERR_HIP (-6)       /* a HIP runtime call failed */
#define MPD_ERR_N (-7)         /* n < 0 or too large */
#define MPD_ERR_RULE (-8)      /* m_max < 0 or u < 0 */

#define MPD_FLAG_FAIL 1u
#define MPD_FLAG_TIMEOUT 2u

/* Message registers are kept as 16-bit emission times of sub-steps, so that
 * v * T_max <= 32767 keeps every register exact (no truncation). */
#define MPD_T_MAX_LIMIT 10922

/* Library version string. */
const char *mpd_version(void);

/* Message of the last failing call on this host thread ("" if none). */
const char *mpd_last_error(void);

/* Bytes of device workspace that a decode of n samples of size L needs
 * (0 if none).  Lattices up to L = 128 decode entirely on chip; from 256 on
 * keep two copies of the per-site state (8 B of registers + 1 bit of
 * syndrome per site) plus per-sample bookkeeping. */
size_t mpd_workspace_bytes(int L, int64_t n);

/* Decode n seeded noise samples of size L at noise strength p.
 *   d_seeds            [n] uint64 seeds (device)
 *   T_max              step budget, 0 <= T_max <= MPD_T_MAX_LIMIT
 *   d_T_dec            [n] int32  decoding time (steps) or T_max on timeout
 *   d_flags            [n] uint8  MPD_FLAG_* bits
 *   d_final_syndrome   [n][ceil(L*L/32)] uint32 anyons after the last step
 *                      (all zero for a decoded sample); may be NULL
 *   d_workspace        >= mpd_workspace_bytes(L, n) bytes, 256-byte aligned
 *                      (may be NULL when that size is 0)
 * Supported L: 3 <= L <= 128 when a strip height H <= 16 divides L with
 * L*L/H <= 1024 threads (every L <= 32, and e.g. 48, 64, 96, 100, 128), and
 * multiples of 16 from 256 to 16384 (at most 65535 samples per call for
 * these, else MPD_ERR_N). */
int mpd_decode_batch(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max,
                     int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_final_syndrome,
                     void *d_workspace, size_t ws_bytes, void *stream);

/* Allocation-free decode, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as mpd_decode_batch without the
 * workspace: the band path (L >= 256) keeps its state in a scratch array of
 * MPD_STATIC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends, and runs its later passes on the device (no host
 * wait, no pinned host memory).  A call whose band-path state would exceed
 * the scratch (mpd_workspace_bytes(L, n) > MPD_STATIC_SCRATCH_BYTES: about
 * 124 samples at L = 256, 31 at L = 512, 7 at L = 1024) fails with
 * MPD_ERR_WORKSPACE and enqueues nothing; lattices up to L = 128 need no
 * scratch.  No call allocates or frees device or pinned host memory (the
 * first call on a device looks the scratch up; with mpd_profile on, timing
 * events are still created).  Every call on one device shares that
 * device's scratch: calls that overlap on a device (several streams or host
 * threads) race and give wrong results; order them on one stream.  The
 * scratch keeps the last call's contents; each call clears what it reads
 * before reading it. */
#define MPD_STATIC_SCRATCH_BYTES (128u << 20)
int mpd_decode_batch_static(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int32_t *d_T_dec,
                            uint8_t *d_flags, uint32_t *d_final_syndrome, void *stream);

/* Decode n explicit error patterns (hand-built cases, exhaustive checks).
 *   d_links            [n][ceil(2*L*L/32)] uint32 link bits (see above)
 * Other arguments as mpd_decode_batch.  Supported L: as mpd_decode_batch;
 * the workspace is needed from L = 256 on (mpd_workspace_bytes(L, n)),
 * where the decode runs the same passes as a seeded one. */
int mpd_decode_errors(int L, const uint32_t *d_links, int64_t n, int T_max, int32_t *d_T_dec,
                      uint8_t *d_flags, uint32_t *d_final_syndrome, void *d_workspace,
                      size_t ws_bytes, void *stream);

/* Run exactly t_exact decoder steps on explicit error patterns, with no early
 * exit, and export the full decoder state (checkpoint / parity debugging).
 *   d_m_out            [n][4][L*L] int16 message registers m^{+x}, m^{-x},
 *                      m^{+y}, m^{-y} after step t_exact (distance form of the
 *                      paper: 0 = no message)
 *   d_sigma_out        [n][ceil(L*L/32)] uint32 anyon bits after step t_exact
 *   d_wind_out         [n] uint8: bit 0 Wx(E), bit 1 Wy(E), bit 2 Wx(C),
 *                      bit 3 Wy(C), winding parities of the error and of the
 *                      correction applied so far, across the cuts x = L-1 and
 *                      y = L-1
 * Supported L: 3 <= L <= 128 (mpd_run_steps_ws takes every size). */
int mpd_run_steps(int L, const uint32_t *d_links, int64_t n, int t_exact, int16_t *d_m_out,
                  uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream);

/* Limited classical memory (Sec. 5.3, the corollary on thresholds with
 * limited memory; message values in {0, ..., m_max} as in Sec. 3.1).
 *   m_max   > 0: an update whose message value would exceed m_max yields 0
 *           (the message disappears); 0: no truncation
 *   u       > 0: at every decoder step t (counted from 1) that is a multiple
 *           of u, every anyon moves one link in a random direction instead of
 *           following its messages (links flip through the same OR rule);
 *           0: no random moves.  Directions: Philox4x32-10 keyed by the
 *           sample's 64-bit seed, counter (i >> 1, t, 0x4D4F5645, 0), word
 *           (i & 1) of site i = y*L + x, mod 4 -> +x, -x, +y, -y.
 * With m_max = u = 0 each call equals its plain counterpart.  The seeds of
 * mpd_decode_rule key both the noise and the random moves; the explicit-
 * error forms take move seeds (may be NULL when u = 0).  MPD_ERR_RULE for
 * m_max < 0 or u < 0; other arguments and errors as the plain calls.  Both
 * band-path drivers support the variant; mixed and learned decodes use the
 * plain rule. */
int mpd_decode_rule(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int m_max, int u,
                    int32_t *d_T_dec, uint8_t *d_flags, uint32_t *d_final_syndrome, void *d_workspace,
                    size_t ws_bytes, void *stream);
int mpd_decode_errors_rule(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n,
                           int T_max, int m_max, int u, int32_t *d_T_dec, uint8_t *d_flags,
                           uint32_t *d_final_syndrome, void *stream);
int mpd_run_steps_rule(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n,
                       int t_exact, int m_max, int u, int16_t *d_m_out, uint32_t *d_sigma_out,
                       uint8_t *d_wind_out, void *stream);

/* Open lattice (the appendix on open boundaries, Def. "message passing
 * automaton with open boundaries"): sites (x, y), 0 <= x, y < L, no wrap.
 * The columns x = 0 and x = L-1 are the rough boundary B: they carry no
 * syndrome and no messages, source x-messages into the bulk (a bulk site
 * next to B reads a message of value 1 from it) and absorb anyons that move
 * onto them.  Rows y = 0 and y = L-1 end smooth (lines are clipped).  The
 * qubits are the links with a bulk endpoint: x-links (x,y)-(x+1,y) for
 * x <= L-2 and y-links (x,y)-(x,y+1) for y <= L-2, 1 <= x <= L-2; noise on,
 * and explicit error bits of, other links are ignored (same link ids and
 * noise words as on the torus).  One logical qubit: flag bit 0 is set iff
 * error + correction crosses the cut between columns L-2 and L-1 an odd
 * number of times, or on timeout.  Final syndromes have no bits at B; the
 * state export reports 0 registers at B, and wind bits 0 (error) and 2
 * (correction) on that cut (bits 1 and 3 are 0).  Supported L: 3..128 (the
 * resident kernel; the explicit-error and state-export forms take only
 * these), and for mpd_decode_open also multiples of 16 from 256 to 16384
 * (the band path, either driver; workspace as for mpd_decode_batch).  Other
 * arguments and errors as the torus calls. */
int mpd_decode_open(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int32_t *d_T_dec,
                    uint8_t *d_flags, uint32_t *d_final_syndrome, void *d_workspace, size_t ws_bytes,
                    void *stream);
int mpd_decode_errors_open(int L, const uint32_t *d_links, int64_t n, int T_max, int32_t *d_T_dec,
                           uint8_t *d_flags, uint32_t *d_final_syndrome, void *stream);
int mpd_run_steps_open(int L, const uint32_t *d_links, int64_t n, int t_exact, int16_t *d_m_out,
                       uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream);

/* Resume the decoder from an exported state (checkpoint / resume): the state
 * mpd_run_steps, mpd_run_steps_rule or this call wrote after t_start steps --
 * registers d_m_in [n][4][L*L] int16 in distance form, syndrome bits
 * d_sigma_in and winding bits d_wind_in (layouts as mpd_run_steps) -- is run
 * for exactly t_exact more steps and exported in the same form.  The result
 * equals mpd_run_steps(t_start + t_exact) on the original errors; with the
 * limited-memory variant (m_max, u; move seeds as mpd_run_steps_rule) the
 * steps keep their absolute numbers t_start + 1, ...  Inputs must be such an
 * export (registers at most 3 t_start); other values give unspecified
 * results but no out-of-bounds access.  Inputs and outputs may be the same
 * buffers (each sample is read completely before it is written).  Torus, L =
 * 3..128 (the resident kernel); t_start + t_exact <= MPD_T_MAX_LIMIT.
 * Errors as mpd_run_steps_rule. */
int mpd_run_steps_from(int L, const int16_t *d_m_in, const uint32_t *d_sigma_in, const uint8_t *d_wind_in, int64_t n,
                       int t_start, int t_exact, int m_max, int u, const uint64_t *d_move_seeds, int16_t *d_m_out,
                       uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream);

/* State export and resume for every supported lattice size (checkpoint /
 * resume, parity debugging), Def. "synchronous automaton decoder": exactly
 * t_exact decoder steps, no early exit.
 *   mpd_run_steps_ws       from explicit errors d_links, as
 *                          mpd_run_steps_rule (m_max, u, move seeds);
 *   mpd_run_steps_from_ws  from a state exported after t_start steps, as
 *                          mpd_run_steps_from.
 * Outputs (d_m_out [n][4][L*L] int16 distance form, d_sigma_out syndrome
 * bits, d_wind_out winding bits) as mpd_run_steps.  Up to L = 128 these are
 * the resident calls and the workspace is ignored; for multiples of 16 from
 * 256 to 16384 the band path runs passes of up to k_first steps over all
 * samples (no compaction) in a workspace of mpd_workspace_bytes(L, n)
 * bytes (256-byte aligned), then converts its state (at most 65535 samples
 * per call, else MPD_ERR_N).  Results equal the resident kernel's and the
 * paper's rule step by step; on the band path the inputs and outputs of the
 * resume form must not overlap.  Errors as mpd_run_steps_rule /
 * mpd_run_steps_from plus MPD_ERR_WORKSPACE. */
int mpd_run_steps_ws(int L, const uint32_t *d_links, const uint64_t *d_move_seeds, int64_t n, int t_exact, int m_max,
                     int u, int16_t *d_m_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *d_workspace,
                     size_t ws_bytes, void *stream);
int mpd_run_steps_from_ws(int L, const int16_t *d_m_in, const uint32_t *d_sigma_in, const uint8_t *d_wind_in,
                          int64_t n, int t_start, int t_exact, int m_max, int u, const uint64_t *d_move_seeds,
                          int16_t *d_m_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *d_workspace,
                          size_t ws_bytes, void *stream);

/* Marching-soldiers desynchronization (Sec. "Desynchronization and
 * Lindbladian dynamics": Def. "marching soldiers desynchronization", Def.
 * "desynchronized decoders", Prop. "faithful Lindbladian simulation") of the
 * plain rule on the torus, 5 <= L <= 64, one workgroup per sample.
 *
 * Each site advances on its own: v = 3 message updates, then one feedback
 * update applying F to its links to (x+1,y) and (x,y+1); t_sim counts them.
 * An update of a site is accepted only if no site within infinity-distance
 * 2 has a smaller t_sim.  Neighbours one update ahead are read through their
 * previous registers, and feedback of step k reads every syndrome without
 * the step-k flips already applied, so the decoder computes exactly what the
 * synchronous one computes, in any update order.
 *
 * Clock: time runs in slots.  In slot s site i rings iff word 2*(i&1) of
 * Philox4x32-10(key = clock seed, counter (i >> 1, s, 0x41535943, 0)) is
 * below floor(rho * 2^32) (at least 1); ringing sites attempt one update
 * each in increasing order of (word 2*(i&1)+1 >> 13, i).  Small rho approaches
 * independent rate-1 Poisson clocks with slots of length rho.
 *
 * mpd_decode_async: noise from d_seeds as mpd_decode_batch (the same seed
 * keys the clock), then run until the syndrome holds no anyon and no flip
 * of any step is pending, or S_max slots.  Outputs per sample:
 *   d_T_async   [n] int32: 1 + the last slot in which a link flipped (0 if
 *               none); times rho is the decoding time in units of the
 *               clocks' mean interval
 *   d_flags     [n] uint8: as mpd_decode_batch; timeout = S_max slots spent
 *               with anyons or pending flips left
 *   d_slots     [n] int32 slots run (may be NULL)
 *   d_updates   [n] int64 accepted updates over all sites (may be NULL)
 *   d_final_syndrome  [n][ceil(L*L/32)] (may be NULL)
 * The correction, the final syndrome and the failure bit equal those of the
 * synchronous decoder with the same seed whenever neither times out.
 *
 * mpd_run_async: explicit error chains (link bit arrays) and clock seeds;
 * runs until every site has made 4 t_target updates (sites that have stop
 * attempting) or S_max slots.  Outputs: d_slots [n] int32; d_updates [n]
 * int64 (may be NULL); d_m_out [n][4][L*L] int16 registers m^new in
 * distance form (order +x, -x, +y, -y); d_tsim_out [n][L*L] uint16; the
 * physical syndrome d_sigma_out as a syndrome bit array; d_wind_out as
 * mpd_run_steps.  Once every site has reached the target these equal
 * mpd_run_steps(t_exact = t_target).
 *
 * Errors: MPD_ERR_L (L outside 5..64), MPD_ERR_P (p outside [0, 1] or rho
 * outside (0, 1]), MPD_ERR_TMAX (S_max outside [0, MPD_ASYNC_SLOT_LIMIT],
 * t_target outside [0, MPD_ASYNC_SLOT_LIMIT / 4]), MPD_ERR_N, MPD_ERR_PTR
 * (required pointer NULL, or any pointer misaligned for its type).  No
 * workspace; no host synchronization. */
#define MPD_ASYNC_SLOT_LIMIT 65000
int mpd_decode_async(int L, double p, const uint64_t *d_seeds, int64_t n, double rho, int S_max, int32_t *d_T_async,
                     uint8_t *d_flags, int32_t *d_slots, int64_t *d_updates, uint32_t *d_final_syndrome,
                     void *stream);
int mpd_run_async(int L, const uint32_t *d_links, const uint64_t *d_clock_seeds, int64_t n, int t_target, double rho,
                  int S_max, int32_t *d_slots, int64_t *d_updates, int16_t *d_m_out, uint16_t *d_tsim_out,
                  uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream);

/* Uncoordinated desynchronization (Sec. "Uncoordinated desynchronization")
 * of the plain rule on the torus, 5 <= L <= 64: the marching-soldiers clock
 * without the lag rule and without old copies.  Every ring applies one update
 * to the site: a message update reads the current registers and syndromes on
 * its lines; a motion update of an anyon site moves that anyon one link along
 * its force (+a for f^a = -1, -a for f^a = +1), annihilating it with an anyon
 * there.  Which updates are motions is set by `schedule`:
 *   MPD_UNCOORD_CYCLIC  every fourth update of a site (v = 3 message updates,
 *                       then one motion, as in the synchronous step);
 *   MPD_UNCOORD_RANDOM  each update independently with probability 1/4:
 *                       word (i & 1) of Philox4x32-10(key = seed, counter
 *                       (i >> 1, slot, 0x54595045, 0)) mod 4 == 3 (messages and
 *                       motion then run on independent Poisson clocks of
 *                       rates 3 and 1 as rho -> 0).
 * This is a different dynamics from the synchronous decoder's: outcomes and
 * decoding times differ.
 *
 * mpd_decode_uncoord: as mpd_decode_async; a decode ends at the first slot
 * boundary with no anyon; d_T_un = 1 + the last slot with a move.
 * mpd_run_uncoord: as mpd_run_async (every site runs 4 t_target updates);
 * t_sim counts all updates.  Arguments, layouts and errors as the
 * marching-soldiers calls; MPD_ERR_N for an unknown schedule. */
#define MPD_UNCOORD_CYCLIC 0
#define MPD_UNCOORD_RANDOM 1
int mpd_decode_uncoord(int L, double p, const uint64_t *d_seeds, int64_t n, double rho, int S_max, int schedule,
                       int32_t *d_T_un, uint8_t *d_flags, int32_t *d_slots, int64_t *d_updates,
                       uint32_t *d_final_syndrome, void *stream);
int mpd_run_uncoord(int L, const uint32_t *d_links, const uint64_t *d_clock_seeds, int64_t n, int t_target,
                    double rho, int S_max, int schedule, int32_t *d_slots, int64_t *d_updates, int16_t *d_m_out,
                    uint16_t *d_tsim_out, uint32_t *d_sigma_out, uint8_t *d_wind_out, void *stream);

/* Temporal blocking of the band path (L >= 256): decoder steps run on chip per
 * pass over HBM, in the first pass (registers still empty) and in later
 * passes.  Results do not depend on it; speed does.  Each value in
 * [1, 15].  L = 0 sets the default for every L and forgets per-L settings;
 * otherwise the setting applies to that L only (defaults 4 and 2).
 * Process-wide, guarded by a mutex. */
int mpd_set_band_schedule(int L, int k_first, int k_next);
int mpd_get_band_schedule(int L, int *k_first, int *k_next);

/* Who drives the later passes of the band path (L >= 256).
 *   MPD_BAND_DRIVER_HOST    one launch per pass; before each, the host reads
 *                           the survivor count back (a wait on the stream)
 *                           and sizes the grid to it, with 4-wave regions
 *                           when the survivors would leave compute units
 *                           idle.  Fastest for a few samples.
 *   MPD_BAND_DRIVER_DEVICE  one persistent launch after the first pass:
 *                           each workgroup takes surviving samples from a
 *                           device list and runs all their passes, tile by
 *                           tile, until each is decoded or reaches T_max.
 *                           No host wait: a band-path decode can then be
 *                           captured into a HIP graph.
 *   MPD_BAND_DRIVER_AUTO    the device on a stream that is being captured,
 *                           else the host.  (After the bit-sliced first
 *                           kernel, see mpd_set_band_bits, the device-driven
 *                           survivors go straight to the persistent launch.)
 * Results never depend on the driver.  L = 0 sets the default and the
 * driver of every per-L setting; otherwise this L only.  A stream under
 * capture always takes the device.  Process-wide, guarded by a mutex;
 * MPD_ERR_N for an unknown driver. */
#define MPD_BAND_DRIVER_AUTO 0
#define MPD_BAND_DRIVER_HOST 1
#define MPD_BAND_DRIVER_DEVICE 2
int mpd_set_band_driver(int L, int driver);
int mpd_get_band_driver(int L, int *driver);

/* First steps of a plain seeded batch in the bit-sliced kernel.  During the
 * first ten decoder steps every emission time is at most 30, so the
 * registers fit in 5-bit planes and a whole torus of L = 64, 128 or 256 fits
 * in one workgroup (L/64 waves; no halo, no HBM state); a sample leaves as
 * soon as it has no anyon.  At L = 256 the others continue on the band path
 * from the state the kernel hands over; at L = 64 and 128 the whole-lattice
 * kernel decodes them again from their seeds (no workspace), so there a
 * batch with one p >= 0.045 (nearly every sample outlives the ten steps)
 * skips the bit-sliced steps; per-sample p always runs them.  Larger
 * lattices run k = min(k_bits, 6) steps in 256 x 256 regions with a halo of
 * 4k (the tiled kernel), then continue on the band path.  k_bits in [0, 10]:
 * the number of such steps (0: the band path's first pass, or the
 * whole-lattice kernel alone).  Applies to mpd_decode_batch,
 * mpd_decode_batch_static, mpd_decode_mixed and the learned decode, with the
 * plain rule (Def. "message passing automaton, general dimensions"); results
 * never depend on it.  L = 0 sets the default and every per-L setting
 * (default 10).  Process-wide, guarded by a mutex; MPD_ERR_TMAX outside
 * [0, 10]. */
int mpd_set_band_bits(int L, int k_bits);
int mpd_get_band_bits(int L, int *k_bits);

/* Autotuner for the band path: decodes the probe batch (same arguments as
 * mpd_decode_batch, outputs overwritten) once per candidate schedule --
 * driver (host, device) x k_first in [1, 8] x k_next in [1, 8], and also
 * the steps of the bit-sliced first kernel (0, 3, 5, 8, 10 at L = 256; 0,
 * 4, 5, 6 of the tiled one above; with it on, k_first is not searched, since
 * the band passes start after it) -- timing each with HIP events on
 * `stream` (a warm-up decode, then a timed one).  The eight fastest are
 * timed again in five interleaved rounds, and the one with the lowest
 * median is kept for this L (mpd_get_band_schedule, mpd_get_band_driver
 * and mpd_get_band_bits then return it).  *k_first, *k_next and *best_ms
 * (that median) receive the choice.  Synchronizes `stream`. */
int mpd_autotune_band(int L, double p, const uint64_t *d_seeds, int64_t n, int T_max, int32_t *d_T_dec,
                      uint8_t *d_flags, void *d_workspace, size_t ws_bytes, void *stream, int *k_first,
                      int *k_next, float *best_ms);

/* Mixed batch: samples of several lattice sizes and per-sample noise
 * strengths in one call.
 *   n_classes, h_L, h_count   host arrays: class c has h_count[c] samples of
 *                             size h_L[c]; samples are ordered by class
 *   d_p, d_seeds              [n] per-sample noise strength and seed
 *   d_T_dec, d_flags          [n] as in mpd_decode_batch
 *   d_final_syndrome          concatenation over classes of
 *                             [h_count[c]][ceil(L_c^2/32)] words; may be NULL
 *   d_workspace               >= mpd_mixed_workspace_bytes(...), 256-byte
 *                             aligned (the sum of the band classes' parts)
 * Classes up to L = 128 run as one launch each on a library-owned side
 * stream forked from `stream` (one workgroup per sample, early exit per
 * sample); larger classes run the band path, each on a library-owned stream
 * with its own part of the workspace, their passes in lockstep (one host wait
 * per round of passes); the call returns after all of them have been joined
 * into `stream`.  When only one class has samples, its decode runs on
 * `stream` itself (no side streams).  Every p in [0, 1]; errors as
 * mpd_decode_batch. */
size_t mpd_mixed_workspace_bytes(int n_classes, const int32_t *h_L, const int64_t *h_count);
int mpd_decode_mixed(int n_classes, const int32_t *h_L, const int64_t *h_count, const double *d_p,
                     const uint64_t *d_seeds, int T_max, int32_t *d_T_dec, uint8_t *d_flags,
                     uint32_t *d_final_syndrome, void *d_workspace, size_t ws_bytes, void *stream);

/* Kernel timing for measurement (not needed for decoding).
 * mpd_profile(1) clears earlier records and starts recording a pair of HIP
 * events on the launch stream around every kernel launch of the library;
 * mpd_profile(0) stops recording (records are kept).  Names: "k_band_noise"
 * (noise and initial syndrome of a band-path batch), "k_band" (one pass of k
 * decoder steps over the bands of L >= 256), "k_bits" (noise and the first
 * steps of an L = 256 batch, bit-sliced), "k_bits_small" (the same at L = 64
 * and 128), "k_bits_tile" (the tiled first steps above L = 256), "k_torus"
 * (whole decode at L = 64 and 128), "k_resident" (whole decode of other
 * small lattices), "k_cnn_forward" and "k_cnn_backward" (decode-time
 * predictor).  Records from several host threads are kept together. */
int mpd_profile(int enable);

/* Sum of the recorded durations (ms) and number of launches of `kernel`;
 * waits for the recorded events to complete. */
int mpd_profile_read(const char *kernel, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------------------
 * Learned scheduling (an addition to the paper's method).
 *
 * A small convolutional network predicts ln(1 + T_dec) of a sample from the
 * anyon counts of its 8 x 8 blocks; a decode can use the prediction to give
 * groups of samples first passes of different depth.  Decoding results never
 * depend on the network: mpd_decode_learned returns exactly what
 * mpd_decode_batch returns for the same seeds.
 *
 * Network, on an M x M map (M = L / 8) of inputs x = count / 8:
 *   layer 1     conv 3x3, 1 -> 16 channels, circular padding, bias, ReLU
 *   layers 2-4  conv 3x3, 16 -> 16, circular padding, bias, ReLU
 *   pooling     global maximum per channel (lowest row-major index on ties)
 *   head        pred = bl + sum_c Wl[c] * feat[c]
 * Convolutions: z[co][y][x] = b[co] + sum over dy, dx in {-1, 0, 1} and ci
 * of W[co][3(dy+1) + (dx+1)][ci] * a[ci][(y+dy) mod M][(x+dx) mod M].
 * Parameters: one float32 vector of MPD_CNN_PARAMS values, in this order:
 *   W1 [16][9] | b1 [16] | W2 [16][9][16] | b2 [16] | W3 | b3 | W4 | b4 |
 *   Wl [16] | bl [1].
 * Arithmetic: conv weights and the activations of layers 1-3 are rounded to
 * bfloat16 (nearest, ties to even), products accumulate in float32 (matrix
 * cores); biases, layer-4 activations, pooling and head are float32.
 * ------------------------------------------------------------------------- */
#define MPD_CNN_PARAMS 7137

/* Anyon counts per 8 x 8 block of seeded samples, uint8 [n][L/8][L/8]
 * (row = block row y/8), for the noise of mpd_decode_batch.  p applies to
 * every sample unless d_p (per-sample [n] double) is given.  L: a multiple
 * of 16 in [16, 16384]. */
int mpd_syndrome_counts(int L, double p, const double *d_p, const uint64_t *d_seeds, int64_t n, uint8_t *d_counts,
                        void *stream);

/* Initial parameters: weights uniform in +-sqrt(6 / fan_in) (He et al.,
 * 2015; fan_in 9, 144, 144, 144, 16), biases 0.  Weight j is
 * (2u - 1) * bound with u = (w + 1/2) / 2^32 in double, rounded to float,
 * where w is word 0 of Philox4x32-10 at counter (j, 0x636e6e31, 0, 0) under
 * key (seed & 0xffffffff, seed >> 32). */
int mpd_cnn_init(float *d_params, uint64_t seed, void *stream);

/* Forward pass on count maps d_counts [n][M][M] (2 <= M <= 2048): d_pred [n]
 * and, if not NULL, d_feat [n][16] (pooled maxima) and d_argmax [n][16]
 * (their row-major positions; NaN and -1 for a channel without a number).
 * Workspace: mpd_cnn_forward_workspace_bytes(M, n) bytes, 256-byte aligned
 * (weights packed for the matrix cores; per-sample maxima when M > 32). */
size_t mpd_cnn_forward_workspace_bytes(int M, int64_t n);
int mpd_cnn_forward(const uint8_t *d_counts, int M, int64_t n, const float *d_params, float *d_pred, float *d_feat,
                    int32_t *d_argmax, void *d_workspace, size_t ws_bytes, void *stream);

/* Training step, part 1: loss = mean over the batch of (pred - target)^2
 * (d_loss [1]) and its gradient with respect to the parameters (d_grad
 * [MPD_CNN_PARAMS], the rounding to bfloat16 taken as the identity); d_pred
 * [n] receives the predictions if not NULL.  2 <= M <= 32, n >= 1.
 * Workspace: mpd_cnn_train_workspace_bytes(M, n) bytes, 256-byte aligned. */
size_t mpd_cnn_train_workspace_bytes(int M, int64_t n);
int mpd_cnn_loss_grad(const uint8_t *d_counts, int M, int64_t n, const float *d_params, const float *d_target,
                      float *d_grad, float *d_loss, float *d_pred, void *d_workspace, size_t ws_bytes,
                      void *stream);

/* Training step, part 2: one Adam update (Kingma and Ba, 2015) of d_params
 * with moments d_m, d_v (all [MPD_CNN_PARAMS] float, zero before step 1);
 * step counts from 1. */
int mpd_cnn_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, int step, float lr, float beta1,
                      float beta2, float eps, void *stream);

/* Decode with learned scheduling: noise and block counts, the network's
 * predictions, then samples with h_edges[b-1] <= pred < h_edges[b] (n_bins
 * groups, 1 <= n_bins <= 8, edges ascending) start with a pass of
 * h_depth[b] steps (1..15); later passes run every survivor at the band
 * schedule's k_next.  p applies to every sample unless d_p (per-sample [n]
 * double, 8-byte aligned) is given; with d_p the results equal those of
 * mpd_decode_mixed with the one class (L, n).  Outputs as mpd_decode_batch,
 * plus d_pred [n] if not NULL.  With one group and d_pred NULL the network
 * is not evaluated: the call is the plain decode with first-pass depth
 * h_depth[0] (the FIFO fallback; d_params is still checked).  With the
 * bit-sliced first kernel on (mpd_set_band_bits), which at L = 256 stops
 * each sample as soon as it has no anyon and above runs the same tiled steps
 * on every sample, the groups set the order in which that kernel takes the
 * samples instead -- the group with the longest predicted decoding time
 * first -- and the depths only have to be valid.  L: a multiple
 * of 16 in [256, 16384], at most 65535 samples.  Workspace:
 * mpd_learned_workspace_bytes(L, n) bytes, 256-byte aligned.  The group
 * sizes stay on the device (each group's first pass is sized there), so
 * the call waits for the host only where mpd_decode_batch does: before the
 * later passes when the host drives them (mpd_set_band_driver).  With the
 * device driver, or on a stream under capture, it never synchronizes and
 * can be captured into a graph. */
size_t mpd_learned_workspace_bytes(int L, int64_t n);
int mpd_decode_learned(int L, double p, const double *d_p, const uint64_t *d_seeds, int64_t n, int T_max,
                       const float *d_params, int n_bins, const float *h_edges, const int *h_depth, int32_t *d_T_dec,
                       uint8_t *d_flags, uint32_t *d_final_syndrome, float *d_pred, void *d_workspace,
                       size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MPD_H */
