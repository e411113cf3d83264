// cnn.hip -- decode-time predictor for learned scheduling (gfx950).
//
// A small convolutional network estimates ln(1 + T_dec) of a noise sample
// from the anyon counts of its 8x8 blocks (an M x M map, M = L / 8); T_dec
// is the decoding time of Def. "logical failure rate, expected decoding
// time, and thresholds" (Sec. 5.1).  The network is not part of the paper:
// it only groups samples by predicted decoding time, and no decoder state or
// result depends on it.
//
// Network (parameter vector of 7137 float32, offsets below):
//   x = count / 8
//   4 x [conv 3x3 with circular padding, bias, ReLU]  (1 -> 16, then 16 -> 16)
//   global max over positions per channel (lowest row-major index on ties)
//   pred = bl + sum_c Wl[c] feat[c]
// Conv weights W[co][tap][ci], tap = 3 (dy + 1) + (dx + 1), read the input
// at (y + dy, x + dx) (a cross-correlation).
//
// Precision: conv weights and the activations of layers 1-3 are bfloat16
// (round to nearest even); products accumulate in float32 on the matrix
// cores; biases, layer-4 activations, the pooling and the head are float32.
// Only non-finite parameters make NaN activations: the row-streamed kernels'
// ReLU (on the bfloat16 bit pattern) passes them on, the whole-map kernel of
// maps below 32 x 32 zeroes them; no decode result depends on either.
//
// Forward: positions form the N dimension of v_mfma_f32_16x16x32_bf16 (16
// positions per instruction), output channels the M dimension and (tap,
// input channel) pairs the K dimension (two taps of 16 channels per
// instruction, five instructions per 3x3 layer).  Activations live in LDS as
// [position][16 channels] bfloat16, so a lane's K slice is one 16-byte read
// and its result (4 channels of one position) one 8-byte write.  Maps up to
// 32 x 32 are processed whole by one workgroup with wrapped indexing (32 x
// 32 maps streamed by rows); wider maps in 32 x 32 output tiles from frames
// with a 4-position halo, also streamed by rows, the per-channel maxima
// meeting in a 64-bit atomic max.
//
// Backward (training, maps up to 32 x 32): the global max routes each
// channel's gradient to a single layer-4 position, so the gradient of a
// sample is the sum of 16 back-propagations through receptive fields of
// 3x3, 5x5, 7x7 and 9x9 positions around those maxima.  One workgroup per
// sample walks them with the layer-1..3 activations stored by the forward
// pass (float32 arithmetic on the vector units) and writes its gradient;
// a reduction kernel sums over the batch in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "engine.h"
#include "host.h"
#include "mpd.h"

namespace mpd {
namespace {

constexpr int CH = 16;
constexpr int OFF_W1 = 0, OFF_B1 = 144;  // W1 [16 co][9 tap]
constexpr int OFF_W2 = 160, OFF_B2 = 2464;
constexpr int OFF_W3 = 2480, OFF_B3 = 4784;
constexpr int OFF_W4 = 4800, OFF_B4 = 7104;
constexpr int OFF_WL = 7120, OFF_BL = 7136;
constexpr int NPARAM = MPD_CNN_PARAMS;
constexpr uint32_t INIT_TAG = 0x636E6E31u;  // second counter word of the initializer
constexpr int WRAP_MAX = 32;                // largest map held whole by one workgroup
constexpr int TILE = 32;                    // output tile of wider maps
constexpr int THREADS_WRAP = 512;
constexpr int BWD_THREADS = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float f) {  // nearest, ties to even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint32_t h) { return __uint_as_float(h << 16); }
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// two floats to packed bfloat16 (lo | hi << 16), nearest-even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}
__device__ __forceinline__ float relu(float z) { return z > 0.f ? z : 0.f; }

// Packed bfloat16 weights in MFMA operand order, built once per forward call
// by k_cnn_prep: Aop[layer][jj][lane] holds the 8 K values of lane `lane`
// for the K block jj (A operand of v_mfma_f32_16x16x32_bf16: row co = lane
// % 16, K = 8 (lane / 16) + 0..7).  Layers 2-4: K block jj covers taps 2jj
// (lane groups 0, 1) and 2jj + 1 (groups 2, 3), 16 input channels each;
// layer 1: K = tap (< 9) in block 0.
constexpr int AOP_UINT4 = 4 * 5 * 64;
// A second packing of layers 2-4 for the row-streaming layers of 32 x 32
// maps (conv_rows32): Arow[layer - 1][lane][2 (dy + 1) + blk] (a lane's six
// blocks are contiguous, so one base address serves them).  Block 0
// holds taps (dy, dx = -1) in K 0..15 and (dy, 0) in K 16..31, block 1 the
// tap (dy, +1) in K 0..15 and zeros, 16 input channels per tap.
constexpr int AROW_UINT4 = 3 * 6 * 64;
constexpr int PREP_UINT4 = AOP_UINT4 + AROW_UINT4;

__global__ void k_cnn_prep(const float *__restrict__ params, uint4 *__restrict__ Aop) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= PREP_UINT4) return;
  if (t >= AOP_UINT4) {
    const int u = t - AOP_UINT4;
    const int layer = 1 + u / 384, lane = (u % 384) / 6, b = u % 6;
    const int co = lane & 15, g = lane >> 4, dy = b / 2 - 1, blk = b & 1;
    const int off = layer == 1 ? OFF_W2 : (layer == 2 ? OFF_W3 : OFF_W4);
    const int dx = blk == 0 ? (g < 2 ? -1 : 0) : 1;
    const bool zero = blk == 1 && g >= 2;
    const int tap = 3 * (dy + 1) + (dx + 1), ci0 = 8 * (g & 1);
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = zero ? 0.f : params[off + (co * 9 + tap) * CH + ci0 + j];
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = pack_bf16(v[2 * j], v[2 * j + 1]);
    Aop[t] = make_uint4(w[0], w[1], w[2], w[3]);
    return;
  }
  const int layer = t / 320, jj = (t / 64) % 5, lane = t % 64;
  const int co = lane & 15, g = lane >> 4;
  float v[8];
  if (layer == 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = jj == 0 ? 8 * g + j : 99;
      v[j] = k < 9 ? params[OFF_W1 + co * 9 + k] : 0.f;
    }
  } else {
    const int off = layer == 1 ? OFF_W2 : (layer == 2 ? OFF_W3 : OFF_W4);
    const int tap = 2 * jj + (g >> 1), ci0 = 8 * (g & 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = tap < 9 ? params[off + (co * 9 + tap) * CH + ci0 + j] : 0.f;
  }
  uint32_t w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = pack_bf16(v[2 * j], v[2 * j + 1]);
  Aop[t] = make_uint4(w[0], w[1], w[2], w[3]);
}

// p / R: a constant division when R is a compile-time constant, else an
// exact float reciprocal (p < 2^20).
__device__ __forceinline__ int row_of(int p, int R) {
  if (__builtin_constant_p(R)) return p / R;
  return (int)(((float)p + 0.5f) * (1.f / (float)R));
}

// Running maximum with the lowest index on ties.
__device__ __forceinline__ void keep_max(float v, int i, float &best, int &bi) {
  // both comparisons evaluated (no short circuit): selects instead of a branch per value
  const bool take = (v > best) | ((v == best) & (i < bi));
  best = take ? v : best;
  bi = take ? i : bi;
}

struct Pool {
  float best[4];
  int idx[4];
};

// Layer geometry: input row stride, output side, output row stride and
// offset.  RtGeom holds them at run time; CtGeom makes them compile-time
// constants (tap offsets then fold into the LDS instructions).
struct RtGeom {
  int S_in, R_out, S_out, out_off;
};
template <int SI, int RO, int SO, int OO>
struct CtGeom {
  static constexpr int S_in = SI, R_out = RO, S_out = SO, out_off = OO;
};

// A operands of one layer for this lane (layer 1 uses block 0 only).  A
// workgroup keeps the current layer's in registers and loads the next
// layer's while it computes (the loads complete during the layer).
struct LayerA {
  bf16x8 A[5];
};
__device__ __forceinline__ void load_layer(const uint4 *__restrict__ Aop, int layer, LayerA &W) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int jj = 0; jj < 5; ++jj)
    W.A[jj] = (layer > 0 || jj == 0) ? __builtin_bit_cast(bf16x8, Aop[layer * 320 + jj * 64 + lane]) : W.A[0];
}
__device__ __forceinline__ void load_biases(const float *__restrict__ P, float *bias_s) {
  if (threadIdx.x < 4 * CH) {
    const int l = threadIdx.x / CH, c = threadIdx.x % CH;
    bias_s[threadIdx.x] = P[(l == 0 ? OFF_B1 : l == 1 ? OFF_B2 : l == 2 ? OFF_B3 : OFF_B4) + c];
  }
}

// One 3x3 layer.  The input buffer has row stride S_in and holds, for
// output position (y, x) (0 <= y, x < R_out), the 3x3 window at rows
// y..y+2 and columns x..x+2 (a border or halo of one position on each
// side).  CIN1: single-channel input [..]; otherwise [..][16].  Outputs go
// to out[(y + o) S_out + x + o][16] (o = out_off); LAST folds them into the
// pooling state instead, with global position ((oy + y) mod M, (ox + x) mod M).
// MONO: a lane meets its global positions in increasing order, so only a
// strictly larger value can replace its running maximum (no tie test).
template <bool CIN1, bool LAST, class G, bool MONO = false>
__device__ __forceinline__ void conv_layer(const uint16_t *__restrict__ in, uint16_t *__restrict__ out, const G &geo,
                                           const bf16x8 *A, const float *__restrict__ b, int M, int oy, int ox,
                                           Pool &pool) {
  const int S_in = geo.S_in, R_out = geo.R_out, S_out = geo.S_out, out_off = geo.out_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  float bias[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bias[r] = b[4 * g + r];
  // this lane's input offset (positions) of each K block: tap 2jj or 2jj + 1
  // (block 4 of lane groups 2, 3 has no tap: it reads tap 8 and zeroes it)
  int toff[5];
#pragma unroll
  for (int jj = 0; jj < 5; ++jj) {
    const int tap = min(2 * jj + (g >> 1), 8);
    toff[jj] = (tap / 3) * S_in + tap % 3;
  }
  const int npos = R_out * R_out, ngroups = (npos + 15) >> 4;
  // Accumulators of one 16-position group (the lane's K slices of its input
  // window times the weights).
  auto group_acc = [&](int p) {
    const int y = row_of(p, R_out);
    const int base = y * S_in + (p - y * R_out);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if (CIN1) {
      u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
      if (g == 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = in[base + (j / 3) * S_in + j % 3];
      } else if (g == 1) {
        v[0] = in[base + 2 * S_in + 2];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], __builtin_bit_cast(bf16x8, v), acc, 0, 0, 0);
    } else {
      uint4 v[5];
#pragma unroll
      for (int jj = 0; jj < 5; ++jj) v[jj] = *reinterpret_cast<const uint4 *>(in + (base + toff[jj]) * CH + 8 * (g & 1));
      if (g >= 2) v[4] = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (int jj = 0; jj < 5; ++jj)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[jj], __builtin_bit_cast(bf16x8, v[jj]), acc, 0, 0, 0);
    }
    return acc;
  };
  // Bias, ReLU, then store (or pool) the lane's 4 channels of position p.
  auto finish = [&](const f32x4 &acc, int p, bool valid) {
    const int y = row_of(p, R_out), x = p - y * R_out;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = relu(acc[r] + bias[r]);
    if (!LAST) {
      if (valid)
        *reinterpret_cast<uint2 *>(out + ((y + out_off) * S_out + x + out_off) * CH + 4 * g) =
            make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
    } else {
      const int gi = ((oy + y) % M) * M + (ox + x) % M;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (MONO) {
          const bool gt = v[r] > pool.best[r];
          pool.best[r] = gt ? v[r] : pool.best[r];
          pool.idx[r] = gt ? gi : pool.idx[r];
        } else {
          keep_max(v[r], gi, pool.best[r], pool.idx[r]);
        }
      }
    }
  };
  // Spare lanes (past the last position) repeat the last position and store nothing.
  for (int grp = wave; grp < ngroups; grp += nwaves) {
    int p1 = (grp << 4) + li;
    const bool v1 = p1 < npos;
    p1 = v1 ? p1 : npos - 1;
    finish(group_acc(p1), p1, v1);
  }
}

// Activations of a whole 32 x 32 map in LDS: [32 rows][33 columns][16
// channels] bfloat16.  Rows and columns wrap by address (no border copies);
// column 32 stays zero and is what the lanes whose second K block holds no
// tap read, so that every lane issues the same loads.
constexpr int M32 = 32, RS32 = (M32 + 1) * CH;  // row stride in bfloat16
constexpr int BUF32 = M32 * RS32;               // one buffer, in bfloat16

// A lane's LDS addresses in the first buffer, fixed for the kernel: wave w
// computes the 16 columns x0 = 16 (w & 1) of output rows y0 .. y0 + 7, y0 =
// 8 (w >> 1), from input rows y0 - 1 .. y0 + 8 (mod 32).  rd[k][b] is the
// lane's K slice of block b in input row y0 - 1 (k = 0), y0 (k = 1; rows up
// to y0 + 7 follow at multiples of RS32) and y0 + 8 (k = 2); block 0 holds
// the tap dx = -1 (lane groups 0, 1) or 0 (groups 2, 3), block 1 dx = +1
// (groups 0, 1) or the zero column.  wr is the lane's output (4 channels)
// in row y0.  The second buffer is the same plus BUF32.
struct Lane32 {
  const uint16_t *rd[3][2];
  uint16_t *wr;
};
__device__ __forceinline__ Lane32 lane32(uint16_t *bufA) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = lane & 15, g = lane >> 4;
  const int x = (wave & 1) * 16 + j, y0 = (wave >> 1) * 8;
  const int col[2] = {(x + M32 - 1 + (g >> 1)) & (M32 - 1), g < 2 ? (x + 1) & (M32 - 1) : M32};
  const int row[3] = {(y0 + M32 - 1) & (M32 - 1), y0, (y0 + 8) & (M32 - 1)};
  Lane32 l;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int b = 0; b < 2; ++b) l.rd[k][b] = bufA + row[k] * RS32 + col[b] * CH + 8 * (g & 1);
  l.wr = bufA + y0 * RS32 + x * CH + 4 * g;
  return l;
}

// K slice of block b in input row y0 - 1 + t (t = 0 .. 9) of the buffer at
// offset IN (0 or BUF32).
template <int IN>
__device__ __forceinline__ uint4 row_slice(const Lane32 &l, int t, int b) {
  const uint16_t *p = t == 0 ? l.rd[0][b] : t == 9 ? l.rd[2][b] : l.rd[1][b] + (t - 1) * RS32;
  return *reinterpret_cast<const uint4 *>(p + IN);
}

// ReLU of two packed bfloat16: a bfloat16's sign is the sign of the same
// bits read as int16, so the maximum with 0 as two int16 (one v_pk_max_i16)
// zeroes the negative ones.  Taken after the rounding, which keeps signs,
// it gives the rounded ReLU; a NaN keeps its bits unless its sign is set.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), s16x2{0, 0}));
}

// Zero column of one buffer (2 x 16 bytes per row).
__device__ __forceinline__ void zero_column32(uint16_t *buf) {
  if (threadIdx.x < 2 * M32)
    reinterpret_cast<uint4 *>(buf + (threadIdx.x >> 1) * RS32 + M32 * CH)[threadIdx.x & 1] = make_uint4(0u, 0u, 0u, 0u);
}

// A 16 -> 16 layer of a whole 32 x 32 map, streamed by rows: the wave walks
// its input rows once; the operand fragment of a row (the taps dx = -1, 0
// in one K block, dx = +1 in a second) serves the three output rows that
// read it (with the weights of dy = -1, 0, +1), which keep three
// accumulators in flight, so each input fragment is read from LDS once for
// three output rows.  The bias is the first instruction's accumulator.  A
// holds the six blocks of Arow for this layer.  IN / OUT: buffer offsets.
// LAST folds the outputs into the pooling state (a lane meets its positions
// in increasing order and starts it at value 0 at its first position: the
// largest ReLU output with the lowest position, found without taking the
// ReLU, since relu(v) > m <=> v > m for m >= 0).
template <bool LAST, int IN, int OUT>
__device__ __forceinline__ void conv_rows32(const Lane32 &l, const bf16x8 *A, const f32x4 &bias, Pool &pool) {
  constexpr int RPW = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = (wave & 1) * 16 + (lane & 15), y0 = (wave >> 1) * RPW;
  if (LAST)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      pool.best[r] = 0.f;
      pool.idx[r] = y0 * M32 + x;
    }
  f32x4 acc[3];
  // fragments of the next input row are loaded one row ahead
  uint4 n0 = row_slice<IN>(l, 0, 0), n1 = row_slice<IN>(l, 0, 1);
#pragma unroll
  for (int t = 0; t < RPW + 2; ++t) {  // input row y0 - 1 + t
    const bf16x8 B0 = __builtin_bit_cast(bf16x8, n0), B1 = __builtin_bit_cast(bf16x8, n1);
    if (t + 1 < RPW + 2) {
      n0 = row_slice<IN>(l, t + 1, 0);
      n1 = row_slice<IN>(l, t + 1, 1);
    }
    // output row u = t - 1 - dy reads this row with the weights of dy
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int u = t - 1 - dy;
      if (u < 0 || u >= RPW) continue;
      f32x4 c = dy == -1 ? bias : acc[u % 3];  // bias: first contribution to row u
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2 * (dy + 1)], B0, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2 * (dy + 1) + 1], B1, c, 0, 0, 0);
      acc[u % 3] = c;
    }
    // row u = t - 2 is complete: ReLU and store, or pool
    if (t >= 2) {
      const int u = t - 2;
      const f32x4 c = acc[u % 3];
      if (!LAST) {
        *reinterpret_cast<uint2 *>(l.wr + OUT + u * RS32) =
            make_uint2(relu_bf16x2(pack_bf16(c[0], c[1])), relu_bf16x2(pack_bf16(c[2], c[3])));
      } else {
        const int gi = (y0 + u) * M32 + x;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bool gt = c[r] > pool.best[r];
          pool.best[r] = gt ? c[r] : pool.best[r];
          pool.idx[r] = gt ? gi : pool.idx[r];
          // update the pooling state here, not after the loop (which would
          // keep every row's accumulators alive)
          asm volatile("" : "+v"(pool.best[r]), "+v"(pool.idx[r]));
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the loads one row ahead, not all hoisted
  }
}

// Layer 1 (one input channel) of a whole 32 x 32 map, streamed by rows as
// conv_rows32, into the first buffer.  T[R][c] (R = 0..33 rows y = R - 1
// mod 32, c = 0..31) holds the inputs at columns c - 1, c, c + 1 (mod 32)
// of that row as four bfloat16 (the last zero).  A lane keeps the triplets
// of the last three rows and assembles the 3 x 3 window of its output
// position as K = tap = 3 (dy + 1) + (dx + 1): K 0..7 in lane group 0, K 8
// in group 1 (the operand layout of the layer-1 block of Aop), so one
// instruction per output row and position group; the bias is its
// accumulator.  Each 32-bit word of the K slice is one byte permutation of
// two triplet words, with per-lane selectors (byte code 12 gives a zero
// byte: the words a lane group does not hold).
__device__ __forceinline__ void conv1_rows32(const uint2 *__restrict__ T, const Lane32 &l, const bf16x8 &A1,
                                             const f32x4 &bias) {
  constexpr int RPW = 8;
  constexpr uint32_t Z = 0x0C0C0C0Cu;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int x0 = (wave & 1) * 16, y0 = (wave >> 1) * RPW;
  // __builtin_amdgcn_perm(hi, lo, sel): byte codes 0..3 pick lo's bytes, 4..7 hi's
  const uint32_t sx = g == 0 ? 0x07060504u : g == 1 ? 0x0C0C0100u : Z;  // r0.x | r2.y low half
  const uint32_t sy = g == 0 ? 0x05040100u : Z;                        // r0.y low half, r1.x low half
  const uint32_t sz = g == 0 ? 0x05040302u : Z;                        // r1.x high half, r1.y low half
  const uint32_t sw = g == 0 ? 0x03020100u : Z;                        // r2.x
  const uint2 *p = T + y0 * M32 + x0 + j;
  uint2 r0, r1 = p[0], r2 = p[M32];  // triplets of rows t - 2, t - 1, t
#pragma unroll
  for (int t = 2; t < RPW + 2; ++t) {
    r0 = r1;
    r1 = r2;
    r2 = p[t * M32];
    // window of output row y0 + t - 2: rows r0 (dy = -1), r1 (0), r2 (+1)
    const uint4 k = make_uint4(__builtin_amdgcn_perm(r0.x, r2.y, sx), __builtin_amdgcn_perm(r1.x, r0.y, sy),
                               __builtin_amdgcn_perm(r1.y, r1.x, sz), __builtin_amdgcn_perm(r2.x, r2.x, sw));
    const f32x4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, __builtin_bit_cast(bf16x8, k), bias, 0, 0, 0);
    *reinterpret_cast<uint2 *>(l.wr + (t - 2) * RS32) =
        make_uint2(relu_bf16x2(pack_bf16(c[0], c[1])), relu_bf16x2(pack_bf16(c[2], c[3])));
  }
}

// One step of a 64-bit (hi, lo) maximum across the lanes of a 16-lane row.
template <int CTRL>
__device__ __forceinline__ void key_step(uint32_t &hi, uint32_t &lo) {
  const uint32_t oh = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, CTRL, 0xF, 0xF, true);
  const uint32_t ol = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, CTRL, 0xF, 0xF, true);
  const bool gt = oh > hi || (oh == hi && ol > lo);
  hi = gt ? oh : hi;
  lo = gt ? ol : lo;
}

// Per-channel (maximum, lowest position) of the pooling state of a
// row-streamed layer 4: every value is >= 0 after the ReLU, so the float
// bits order like the values, and the key (bits << 32 | ~position) has its
// maximum at the largest value with the lowest position.  The 16 lanes of a
// row (one channel group, 16 positions) reduce with DPP row shifts; lane 15
// of each row leaves its four keys in keys[wave][16]; threads 0..15 then
// reduce over the waves.
__device__ __forceinline__ void pool_keys_reduce(const Pool &pool, unsigned long long *keys, float &best, int &bi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    uint32_t hi = __float_as_uint(pool.best[r]), lo = ~(uint32_t)pool.idx[r];
    key_step<0x111>(hi, lo);  // row_shr:1, 2, 4, 8; lanes below the shift read 0 (bound_ctrl)
    key_step<0x112>(hi, lo);
    key_step<0x114>(hi, lo);
    key_step<0x118>(hi, lo);
    if ((lane & 15) == 15) keys[wave * CH + 4 * (lane >> 4) + r] = ((unsigned long long)hi << 32) | lo;
  }
  __syncthreads();
  best = -1.f;
  bi = 0x7FFFFFFF;
  if (threadIdx.x < CH) {
    unsigned long long m = 0ull;
    for (int w = 0; w < nwaves; ++w) m = max(m, keys[w * CH + threadIdx.x]);
    best = __uint_as_float((uint32_t)(m >> 32));
    bi = (int)~(uint32_t)m;
  }
}

// Operands of one row-streamed layer (layer 1..3 = network layers 2..4).
struct LayerRow {
  bf16x8 A[6];
};
__device__ __forceinline__ void load_layer_rows(const uint4 *__restrict__ Arow, int layer, LayerRow &W) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int b = 0; b < 6; ++b) W.A[b] = __builtin_bit_cast(bf16x8, Arow[(layer - 1) * 384 + lane * 6 + b]);
}

// Wrapped border of a [(M+2)^2][16] buffer: row 0 / M+1 and column 0 / M+1
// copy the opposite interior edge.
__device__ __forceinline__ void fill_border(uint16_t *buf, int M) {
  const int S = M + 2, nb = 4 * (M + 1);
  uint4 *u = reinterpret_cast<uint4 *>(buf);
  for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) {
    const int c = i >> 1, half = i & 1;
    int r, q;  // border cell (r, q)
    if (c < M + 2) {
      r = 0;
      q = c;
    } else if (c < 2 * (M + 2)) {
      r = M + 1;
      q = c - (M + 2);
    } else if (c < 2 * (M + 2) + M) {
      r = c - 2 * (M + 2) + 1;
      q = 0;
    } else {
      r = c - 2 * (M + 2) - M + 1;
      q = M + 1;
    }
    const int sr = r == 0 ? M : (r == M + 1 ? 1 : r), sq = q == 0 ? M : (q == M + 1 ? 1 : q);
    u[(r * S + q) * 2 + half] = u[(sr * S + sq) * 2 + half];
  }
}

struct FwdArgs {
  const uint8_t *counts;  // [n][M][M]
  int M;
  int ntile;              // tiles per side (tiled mode)
  const uint4 *Aop;       // packed weights (k_cnn_prep)
  const float *params;
  float *pred;            // [n]
  float *feat;            // [n][16] or null
  int32_t *argmax;        // [n][16] or null
  uint16_t *store;        // [3][n][M*M][16] layer 1-3 activations, or null (whole maps only)
  unsigned long long *pool;  // tiled mode: [n][16] packed maxima, zero on entry
  int64_t n;
};

// Interior of a bordered [(M+2)^2][16] buffer to [M*M][16] in HBM.
__device__ __forceinline__ void store_interior(const uint16_t *src, uint16_t *dst, int M) {
  const uint4 *s = reinterpret_cast<const uint4 *>(src);
  uint4 *d = reinterpret_cast<uint4 *>(dst);
  for (int i = threadIdx.x; i < 2 * M * M; i += blockDim.x) {
    const int pos = i >> 1, y = pos / M, x = pos - y * M;
    d[i] = s[((y + 1) * (M + 2) + x + 1) * 2 + (i & 1)];
  }
}

// A [32][33][16] buffer's 32 x 32 positions to [M*M][16] in HBM.
__device__ __forceinline__ void store_rows32(const uint16_t *src, uint16_t *dst) {
  uint4 *d = reinterpret_cast<uint4 *>(dst);
  for (int i = threadIdx.x; i < 2 * M32 * M32; i += blockDim.x) {
    const int pos = i >> 1, y = pos / M32, x = pos - y * M32;
    d[i] = reinterpret_cast<const uint4 *>(src + y * RS32 + x * CH)[i & 1];
  }
}

// Reduction of the per-lane pooling state to per-channel (max, index) in
// threads 0..15 (returned through `best`, `bi`).
__device__ __forceinline__ void pool_reduce(Pool &pool, float *red_v, int *red_i, float &best, int &bi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
#pragma unroll
  for (int s = 1; s < 16; s <<= 1)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float ov = __shfl_xor(pool.best[r], s);
      const int oi = __shfl_xor(pool.idx[r], s);
      keep_max(ov, oi, pool.best[r], pool.idx[r]);
    }
  if ((lane & 15) == 0)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red_v[wave * CH + 4 * (lane >> 4) + r] = pool.best[r];
      red_i[wave * CH + 4 * (lane >> 4) + r] = pool.idx[r];
    }
  __syncthreads();
  best = -1.f;
  bi = 0x7FFFFFFF;
  if (threadIdx.x < CH)
    for (int w = 0; w < nwaves; ++w) keep_max(red_v[w * CH + threadIdx.x], red_i[w * CH + threadIdx.x], best, bi);
  if (bi == 0x7FFFFFFF) {  // no number in the channel (NaN activations)
    best = __builtin_nanf("");
    bi = -1;
  }
}

__device__ __forceinline__ float head(const float *__restrict__ params, const float *feat) {
  float acc = params[OFF_BL];
  for (int c = 0; c < CH; ++c) acc = fmaf(params[OFF_WL + c], feat[c], acc);
  return acc;
}

__device__ __forceinline__ void pool_init(Pool &pool) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    pool.best[r] = -1.f;
    pool.idx[r] = 0x7FFFFFFF;
  }
}

// Whole map per workgroup (M < 32; 32 x 32 maps take k_cnn_forward32),
// buffers with a wrapped border of one position.  LDS: x [(M+2)^2] | A, B
// [(M+2)^2][16] | pooling.  MC > 0: the map side as a compile-time
// constant, 0: at run time.
template <int MC>
__global__ __launch_bounds__(THREADS_WRAP) __attribute__((amdgpu_waves_per_eu(4))) void k_cnn_forward_wrap(
    FwdArgs a) {  // 4 waves per SIMD: two workgroups per CU, as the LDS allows
  extern __shared__ __align__(16) unsigned char smem[];
  const int M = MC > 0 ? MC : a.M, S = M + 2, SS = S * S;
  using Geo = typename std::conditional<(MC > 0), CtGeom<MC + 2, MC, MC + 2, 1>, RtGeom>::type;
  using GeoL = typename std::conditional<(MC > 0), CtGeom<MC + 2, MC, 0, 0>, RtGeom>::type;
  Geo geo;
  GeoL geol;
  if constexpr (MC == 0) {
    geo = RtGeom{S, M, S, 1};
    geol = RtGeom{S, M, 0, 0};
  }
  uint16_t *xin = reinterpret_cast<uint16_t *>(smem);
  uint16_t *bufA = xin + ((SS + 7) & ~7);
  uint16_t *bufB = bufA + SS * CH;
  float *red_v = reinterpret_cast<float *>(bufB + SS * CH);
  int *red_i = reinterpret_cast<int *>(red_v + (blockDim.x >> 6) * CH);
  __shared__ float feat_s[CH];
  __shared__ float bias_s[4 * CH];
  const float *P = a.params;
  load_biases(P, bias_s);
  LayerA Wc, Wn;  // current and next layer's operands
  load_layer(a.Aop, 0, Wc);
  const size_t act = (size_t)M * M * CH;
  // a fixed grid walks the samples
  for (int64_t s = blockIdx.x; s < a.n; s += gridDim.x) {
    const uint8_t *cnt = a.counts + s * M * M;
    for (int i = threadIdx.x; i < SS; i += blockDim.x) {
      const int r = i / S, q = i - r * S;
      const int y = r == 0 ? M - 1 : (r == M + 1 ? 0 : r - 1), x = q == 0 ? M - 1 : (q == M + 1 ? 0 : q - 1);
      xin[i] = to_bf16((float)cnt[y * M + x] * 0.125f);
    }
    __syncthreads();
    Pool pool;
    pool_init(pool);
    load_layer(a.Aop, 1, Wn);
    conv_layer<true, false>(xin, bufA, geo, Wc.A, bias_s, M, 0, 0, pool);
    Wc = Wn;
    load_layer(a.Aop, 2, Wn);
    __syncthreads();
    fill_border(bufA, M);
    if (a.store) store_interior(bufA, a.store + (size_t)s * act, M);
    __syncthreads();
    conv_layer<false, false>(bufA, bufB, geo, Wc.A, bias_s + CH, M, 0, 0, pool);
    Wc = Wn;
    load_layer(a.Aop, 3, Wn);
    __syncthreads();
    fill_border(bufB, M);
    if (a.store) store_interior(bufB, a.store + ((size_t)a.n + s) * act, M);
    __syncthreads();
    conv_layer<false, false>(bufB, bufA, geo, Wc.A, bias_s + 2 * CH, M, 0, 0, pool);
    Wc = Wn;
    load_layer(a.Aop, 0, Wn);
    __syncthreads();
    fill_border(bufA, M);
    if (a.store) store_interior(bufA, a.store + ((size_t)2 * a.n + s) * act, M);
    __syncthreads();
    conv_layer<false, true, GeoL, true>(bufA, nullptr, geol, Wc.A, bias_s + 3 * CH, M, 0, 0, pool);
    Wc = Wn;
    float best;
    int bi;
    pool_reduce(pool, red_v, red_i, best, bi);
    if (threadIdx.x < CH) {
      feat_s[threadIdx.x] = best;
      if (a.feat) a.feat[s * CH + threadIdx.x] = best;
      if (a.argmax) a.argmax[s * CH + threadIdx.x] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) a.pred[s] = head(P, feat_s);
  }
}

// Whole 32 x 32 maps (L = 256): one workgroup of 8 waves per map, two
// workgroups per CU, a fixed grid walking the maps.  Every layer is
// streamed by rows (conv1_rows32, conv_rows32) over [32][33][16] buffers
// that wrap by address.  The next map's counts are fetched into registers
// while the current map's last layer runs.  LDS: A, B [32][33][16]
// bfloat16 (layer 1's tap triplets and the staged counts live in B until
// layer 2 writes it; B's zero column is cleared again after layer 1) |
// per-wave pooling keys.
__global__ __launch_bounds__(THREADS_WRAP) __attribute__((amdgpu_waves_per_eu(4))) void k_cnn_forward32(FwdArgs a) {
  constexpr int M = M32, S = M + 2;
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t *bufA = reinterpret_cast<uint16_t *>(smem);
  uint16_t *bufB = bufA + BUF32;
  uint2 *T = reinterpret_cast<uint2 *>(bufB);                        // [34][32] layer-1 tap triplets
  uint16_t *stage = reinterpret_cast<uint16_t *>(T + S * M);         // [M*M/2] staged counts (2 per entry)
  unsigned long long *pool_keys = reinterpret_cast<unsigned long long *>(bufB + BUF32);  // [NW][16]
  __shared__ float feat_s[CH];
  __shared__ float bias_s[4 * CH];
  __shared__ float head_s[CH + 1];
  const float *P = a.params;
  load_biases(P, bias_s);
  if (threadIdx.x <= CH) head_s[threadIdx.x] = P[OFF_WL + threadIdx.x];  // Wl[16], then bl
  zero_column32(bufA);  // B's is cleared per map, after its tap triplets are used
  const int lane = threadIdx.x & 63;
  const Lane32 l = lane32(bufA);
  const size_t act = (size_t)M * M * CH;
  // this thread's two counts of the first map (M*M/2 = THREADS_WRAP pairs)
  uint16_t nxt = 0;
  if ((int64_t)blockIdx.x < a.n) nxt = reinterpret_cast<const uint16_t *>(a.counts + blockIdx.x * M * M)[threadIdx.x];
  __syncthreads();  // biases
  f32x4 bias[4];  // per layer: this lane's four output channels
#pragma unroll
  for (int k = 0; k < 4; ++k)
    bias[k] = f32x4{bias_s[k * CH + 4 * (lane >> 4)], bias_s[k * CH + 4 * (lane >> 4) + 1],
                    bias_s[k * CH + 4 * (lane >> 4) + 2], bias_s[k * CH + 4 * (lane >> 4) + 3]};
  for (int64_t s = blockIdx.x; s < a.n; s += gridDim.x) {
    stage[threadIdx.x] = nxt;
    __syncthreads();
    {  // tap triplets of layer 1: T[R][c] = x at columns c - 1 .. c + 1 of row R - 1 (mod M)
      const uint8_t *cs = reinterpret_cast<const uint8_t *>(stage);
      for (int i = threadIdx.x; i < S * M; i += blockDim.x) {
        const int R = i / M, c = i - R * M, y = (R + M - 1) % M;
        const float u0 = (float)cs[y * M + (c + M - 1) % M], u1 = (float)cs[y * M + c],
                    u2 = (float)cs[y * M + (c + 1) % M];
        T[i] = make_uint2(pack_bf16(u0 * 0.125f, u1 * 0.125f), pack_bf16(u2 * 0.125f, 0.f));
      }
    }
    __syncthreads();
    // The operand base is opaque per map (it stays in scalar registers), so
    // that the compiler does not hoist one 64-bit address per operand block
    // out of the loop.
    const uint4 *Aop = a.Aop;
    asm volatile("" : "+s"(Aop));
    const uint4 *Arow = Aop + AOP_UINT4;
    LayerRow Wr;
    conv1_rows32(T, l, __builtin_bit_cast(bf16x8, Aop[lane]), bias[0]);
    Pool pool;  // set by the last layer
    load_layer_rows(Arow, 1, Wr);
    __syncthreads();
    zero_column32(bufB);  // read first by layer 3, after the next barrier
    if (a.store) store_rows32(bufA, a.store + (size_t)s * act);
    conv_rows32<false, 0, BUF32>(l, Wr.A, bias[1], pool);
    load_layer_rows(Arow, 2, Wr);
    __syncthreads();
    if (a.store) store_rows32(bufB, a.store + ((size_t)a.n + s) * act);
    conv_rows32<false, BUF32, 0>(l, Wr.A, bias[2], pool);
    load_layer_rows(Arow, 3, Wr);
    __syncthreads();
    if (a.store) store_rows32(bufA, a.store + ((size_t)2 * a.n + s) * act);
    if (s + gridDim.x < a.n) nxt = reinterpret_cast<const uint16_t *>(a.counts + (s + gridDim.x) * M * M)[threadIdx.x];
    conv_rows32<true, 0, 0>(l, Wr.A, bias[3], pool);
    float best;
    int bi;
    pool_keys_reduce(pool, pool_keys, best, bi);
    if (threadIdx.x < CH) {
      feat_s[threadIdx.x] = best;
      if (a.feat) a.feat[s * CH + threadIdx.x] = best;
      if (a.argmax) a.argmax[s * CH + threadIdx.x] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float acc = head_s[CH];
      for (int c = 0; c < CH; ++c) acc = fmaf(head_s[c], feat_s[c], acc);
      a.pred[s] = acc;
    }
  }
}

// Wider maps (M > 32), row-streamed like k_cnn_forward32: 32 x 32 output
// tiles, each from a frame of map rows ty0 - 5 .. ty0 + 36 and columns
// tx0 - 4 .. tx0 + 45 (wrapping mod M).  12 waves: three 16-column groups x
// four bands of 10 rows.  Layers 1-3 compute frame rows 0..39 and columns
// 1..48 into [42 rows][51 columns][16] buffers (row index = frame row + 1;
// column 50 stays zero for the lanes with no second K block); layer 4
// computes frame rows and columns 4..35 (8 waves: two column groups x four
// bands of 8 rows).  Outputs a layer computes outside its valid region
// (layer 1: all of its rows and columns, layer l >= 2: frame rows l - 1 ..
// 40 - l, columns l .. 49 - l) read buffer rows or columns nobody wrote; they
// only feed outputs that are outside the valid region too, so layer 4's
// outputs are those of the whole map at the tile's positions.
constexpr int RT_NW = 12;                 // waves per workgroup
constexpr int RT_BR = 10;                 // output rows per wave (layers 1-3)
constexpr int RT_COLS = 51;               // activation columns: frame columns 0..49, zero column 50
constexpr int RT_Z = 50;                  // the zero column
constexpr int RT_RS = RT_COLS * CH;       // row stride in bfloat16
constexpr int RT_ROWS = TILE + 10;        // activation rows: frame rows -1..40
constexpr int RT_BUF = RT_ROWS * RT_RS;   // one buffer, in bfloat16
constexpr int RT_TC = 48;                 // tap-triplet columns (frame columns 1..48)
constexpr int RT_XC = RT_TC + 2;          // staged count columns (frame columns 0..49)

size_t rtile_lds() {  // A, B, per-wave pooling results (floats and indices)
  return (size_t)2 * RT_BUF * 2 + (size_t)RT_NW * CH * 8;
}

// Zero column of one [RT_ROWS][RT_COLS][16] buffer.
__device__ __forceinline__ void zero_column_rt(uint16_t *buf) {
  for (int i = threadIdx.x; i < 2 * RT_ROWS; i += blockDim.x)
    reinterpret_cast<uint4 *>(buf + (i >> 1) * RT_RS + RT_Z * CH)[i & 1] = make_uint4(0u, 0u, 0u, 0u);
}

// One row-streamed 16 -> 16 layer over NR output rows of one wave (see
// conv_rows32).  rd[b]: the lane's K slice of block b in the input row above
// its first output row; wr: its output (4 channels) in its first output
// row.  LAST folds the outputs into the pooling state instead: the output
// in row u is at map position ((my0 + u) mod M, mx).
template <int NR, bool LAST>
__device__ __forceinline__ void conv_rows_rt(const uint16_t *rd0, const uint16_t *rd1, uint16_t *wr,
                                             const bf16x8 *A, const f32x4 &bias, Pool &pool, int my0, int mx,
                                             int M) {
  f32x4 acc[3];
  uint4 n0 = *reinterpret_cast<const uint4 *>(rd0), n1 = *reinterpret_cast<const uint4 *>(rd1);
  int my = my0;
#pragma unroll
  for (int t = 0; t < NR + 2; ++t) {  // input row t - 1 relative to the first output row
    const bf16x8 B0 = __builtin_bit_cast(bf16x8, n0), B1 = __builtin_bit_cast(bf16x8, n1);
    if (t + 1 < NR + 2) {
      n0 = *reinterpret_cast<const uint4 *>(rd0 + (t + 1) * RT_RS);
      n1 = *reinterpret_cast<const uint4 *>(rd1 + (t + 1) * RT_RS);
    }
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int u = t - 1 - dy;
      if (u < 0 || u >= NR) continue;
      f32x4 c = dy == -1 ? bias : acc[u % 3];  // bias: first contribution to row u
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2 * (dy + 1)], B0, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2 * (dy + 1) + 1], B1, c, 0, 0, 0);
      acc[u % 3] = c;
    }
    if (t >= 2) {
      const int u = t - 2;
      const f32x4 c = acc[u % 3];
      if (!LAST) {
        *reinterpret_cast<uint2 *>(wr + u * RT_RS) =
            make_uint2(relu_bf16x2(pack_bf16(c[0], c[1])), relu_bf16x2(pack_bf16(c[2], c[3])));
      } else {
        const int gi = my * M + mx;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          keep_max(relu(c[r]), gi, pool.best[r], pool.idx[r]);
          asm volatile("" : "+v"(pool.best[r]), "+v"(pool.idx[r]));
        }
        my = my + 1 == M ? 0 : my + 1;
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the loads one row ahead, not all hoisted
  }
}

__global__ __launch_bounds__(RT_NW * 64) void k_cnn_forward_rtile(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M = a.M;
  uint16_t *bufA = reinterpret_cast<uint16_t *>(smem);
  uint16_t *bufB = bufA + RT_BUF;
  uint2 *T = reinterpret_cast<uint2 *>(bufB);                         // [RT_ROWS][RT_TC] layer-1 tap triplets
  uint8_t *xs = reinterpret_cast<uint8_t *>(T + RT_ROWS * RT_TC);     // [RT_ROWS][RT_XC] staged counts
  float *red_v = reinterpret_cast<float *>(bufB + RT_BUF);
  int *red_i = reinterpret_cast<int *>(red_v + RT_NW * CH);
  __shared__ float bias_s[4 * CH];
  load_biases(a.params, bias_s);
  zero_column_rt(bufA);  // B's is cleared per item, after its tap triplets are used
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = lane & 15, g = lane >> 4;
  // layers 1-3: column group gc, rows RT_BR b .. RT_BR b + RT_BR - 1 (frame)
  const int gc = wave % 3, b = wave / 3;
  const int fc = 1 + 16 * gc + j, fr0 = RT_BR * b;
  const int c0 = fc - 1 + (g >> 1), c1 = g < 2 ? fc + 1 : RT_Z;
  const int rdo0 = fr0 * RT_RS + c0 * CH + 8 * (g & 1), rdo1 = fr0 * RT_RS + c1 * CH + 8 * (g & 1);
  const int wro = (fr0 + 1) * RT_RS + fc * CH + 4 * g;
  __syncthreads();  // biases
  // this lane's four output channels of layer l's bias (read per layer: few registers stay live)
  auto bias = [&](int l) { return *reinterpret_cast<const f32x4 *>(bias_s + l * CH + 4 * g); };
  const int nt = a.ntile;
  const int64_t items = a.n * nt * nt;
  const uint4 *Arow = a.Aop + AOP_UINT4;
  // This thread's counts of an item's frame (rows -1..40, i.e. map rows
  // ty0 - 5 .., and columns 0..49): entries threadIdx.x + k blockDim.x.
  // The next item's are fetched while the current one's last layer runs.
  constexpr int XPT = (RT_ROWS * RT_XC + RT_NW * 64 - 1) / (RT_NW * 64);
  uint8_t pre[XPT];
  auto fetch = [&](int64_t item) {
    const int tt = (int)(item % (nt * nt));
    const int ty0 = (tt / nt) * TILE, tx0 = (tt % nt) * TILE;
    const uint8_t *cnt = a.counts + (item / (nt * nt)) * M * M;
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int i = threadIdx.x + k * RT_NW * 64;
      if (i < RT_ROWS * RT_XC) {
        const int R = i / RT_XC, C = i - R * RT_XC;
        int y = ty0 - 5 + R, x = tx0 - 4 + C;  // in [-5, M + 45): at most two wraps for M >= 34
        y += y < 0 ? M : 0;
        x += x < 0 ? M : 0;
        y -= y >= M ? M : 0;
        x -= x >= M ? M : 0;
        y -= y >= M ? M : 0;
        x -= x >= M ? M : 0;
        pre[k] = cnt[y * M + x];
      }
    }
  };
  if ((int64_t)blockIdx.x < items) fetch(blockIdx.x);
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t s = it / (nt * nt);
    const int t = (int)(it % (nt * nt));
    const int ty0 = (t / nt) * TILE, tx0 = (t % nt) * TILE;
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int i = threadIdx.x + k * RT_NW * 64;
      if (i < RT_ROWS * RT_XC) xs[i] = pre[k];
    }
    __syncthreads();
    // tap triplets: T[R][k] = x at frame columns k, k + 1, k + 2 of frame row R - 1
    for (int i = threadIdx.x; i < RT_ROWS * RT_TC; i += blockDim.x) {
      const int R = i / RT_TC, k = i - R * RT_TC;
      const uint8_t *q = xs + R * RT_XC + k;
      T[i] = make_uint2(pack_bf16((float)q[0] * 0.125f, (float)q[1] * 0.125f), pack_bf16((float)q[2] * 0.125f, 0.f));
    }
    __syncthreads();
    {  // layer 1: output rows fr0 .. fr0 + RT_BR - 1, column fc; K = tap as in conv1_rows32
      constexpr uint32_t Z = 0x0C0C0C0Cu;
      const uint32_t sx = g == 0 ? 0x07060504u : g == 1 ? 0x0C0C0100u : Z;
      const uint32_t sy = g == 0 ? 0x05040100u : Z;
      const uint32_t sz = g == 0 ? 0x05040302u : Z;
      const uint32_t sw = g == 0 ? 0x03020100u : Z;
      const bf16x8 A1 = __builtin_bit_cast(bf16x8, a.Aop[lane]);
      const uint2 *p = T + fr0 * RT_TC + fc - 1;
      uint16_t *w1 = bufA + wro;
      uint2 r0, r1 = p[0], r2 = p[RT_TC];
#pragma unroll
      for (int tt = 2; tt < RT_BR + 2; ++tt) {
        r0 = r1;
        r1 = r2;
        r2 = p[tt * RT_TC];
        const uint4 k = make_uint4(__builtin_amdgcn_perm(r0.x, r2.y, sx), __builtin_amdgcn_perm(r1.x, r0.y, sy),
                                   __builtin_amdgcn_perm(r1.y, r1.x, sz), __builtin_amdgcn_perm(r2.x, r2.x, sw));
        const f32x4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, __builtin_bit_cast(bf16x8, k), bias(0), 0, 0, 0);
        *reinterpret_cast<uint2 *>(w1 + (tt - 2) * RT_RS) =
            make_uint2(relu_bf16x2(pack_bf16(c[0], c[1])), relu_bf16x2(pack_bf16(c[2], c[3])));
      }
    }
    LayerRow Wr;
    load_layer_rows(Arow, 1, Wr);
    Pool pool;
    pool_init(pool);
    __syncthreads();
    zero_column_rt(bufB);  // read first by layer 3, after the next barrier
    conv_rows_rt<RT_BR, false>(bufA + rdo0, bufA + rdo1, bufB + wro, Wr.A, bias(1), pool, 0, 0, M);
    load_layer_rows(Arow, 2, Wr);
    __syncthreads();
    conv_rows_rt<RT_BR, false>(bufB + rdo0, bufB + rdo1, bufA + wro, Wr.A, bias(2), pool, 0, 0, M);
    load_layer_rows(Arow, 3, Wr);
    __syncthreads();
    if (it + gridDim.x < items) fetch(it + gridDim.x);  // after the last weight load: no wait on it before
    if (wave < 8) {  // layer 4: column group gc4, rows 4 + 8 b4 .. 11 + 8 b4 (frame)
      const int gc4 = wave & 1, b4 = wave >> 1;
      const int fc4 = 4 + 16 * gc4 + j, fr4 = 4 + 8 * b4;
      const int c04 = fc4 - 1 + (g >> 1), c14 = g < 2 ? fc4 + 1 : RT_Z;
      const int rd4o0 = fr4 * RT_RS + c04 * CH + 8 * (g & 1), rd4o1 = fr4 * RT_RS + c14 * CH + 8 * (g & 1);
      int my0 = ty0 - 4 + fr4, mx = tx0 - 4 + fc4;  // in [0, M + 36): at most two wraps
      my0 -= my0 >= M ? M : 0;
      mx -= mx >= M ? M : 0;
      my0 -= my0 >= M ? M : 0;
      mx -= mx >= M ? M : 0;
      conv_rows_rt<8, true>(bufA + rd4o0, bufA + rd4o1, nullptr, Wr.A, bias(3), pool, my0, mx, M);
    }
    float best;
    int bi;
    pool_reduce(pool, red_v, red_i, best, bi);
    if (threadIdx.x < CH && bi >= 0) {
      // non-negative floats order as their bit patterns; ties keep the lowest index
      const unsigned long long key =
          ((unsigned long long)__float_as_uint(best) << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)bi);
      atomicMax(&a.pool[s * CH + threadIdx.x], key);
    }
    __syncthreads();  // LDS reused by the next item
  }
}

__global__ void k_cnn_head(FwdArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n) return;
  float feat[CH];
  for (int c = 0; c < CH; ++c) {
    const unsigned long long key = a.pool[s * CH + c];  // 0: no tile had a number
    feat[c] = key ? __uint_as_float((uint32_t)(key >> 32)) : __builtin_nanf("");
    if (a.feat) a.feat[s * CH + c] = feat[c];
    if (a.argmax) a.argmax[s * CH + c] = key ? (int32_t)(0xFFFFFFFFu - (uint32_t)key) : -1;
  }
  a.pred[s] = head(a.params, feat);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Backward (maps up to 32 x 32)
// ---------------------------------------------------------------------------

struct BwdArgs {
  const uint8_t *counts;   // [n][M][M]
  int M;
  int64_t n;
  const float *params;
  const uint16_t *store;   // [3][n][M*M][16]
  const float *feat;       // [n][16]
  const int32_t *argmax;   // [n][16]
  const float *pred;       // [n]
  const float *target;     // [n]
  float *part;             // [n][NPARAM] per-sample gradient of the batch-mean loss
};

// window of radius R around P (offsets -R..R), position index of offset (oy, ox)
__device__ __forceinline__ int wpos(int P, int oy, int ox, int M) {
  int y = P / M + oy, x = P % M + ox;
  y += y < 0 ? M : 0;
  y -= y >= M ? M : 0;
  x += x < 0 ? M : 0;
  x -= x >= M ? M : 0;
  return y * M + x;
}

__global__ __launch_bounds__(BWD_THREADS) void k_cnn_backward(BwdArgs a) {
  // LDS (float): W2, W3, W4 [16][9][16]; W1 [16][9]; windows; dz; accumulators
  __shared__ float W2[2304], W3[2304], W4[2304], W1[144];
  __shared__ float a3w[9 * CH], a2w[25 * CH], a1w[49 * CH], xw[81];
  __shared__ float dz3[9 * CH], dz2[25 * CH], dz1[49 * CH];
  __shared__ float gW1[144], gB1[CH], gW2[2304], gB2[CH], gW3[2304], gB3[CH], gW4[2304], gB4[CH];
  const int tid = threadIdx.x;
  const int64_t s = blockIdx.x;
  const int M = a.M, MM = M * M;
  const float *P = a.params;
  for (int i = tid; i < 2304; i += BWD_THREADS) {  // weights as the forward used them (bfloat16)
    W2[i] = from_bf16(to_bf16(P[OFF_W2 + i]));
    W3[i] = from_bf16(to_bf16(P[OFF_W3 + i]));
    W4[i] = from_bf16(to_bf16(P[OFF_W4 + i]));
    gW2[i] = gW3[i] = gW4[i] = 0.f;
  }
  if (tid < 144) {
    W1[tid] = from_bf16(to_bf16(P[OFF_W1 + tid]));
    gW1[tid] = 0.f;
  }
  if (tid < CH) gB1[tid] = gB2[tid] = gB3[tid] = gB4[tid] = 0.f;
  const float dpred = 2.f * (a.pred[s] - a.target[s]) / (float)a.n;
  const size_t act = (size_t)MM * CH;
  const uint16_t *A1 = a.store + (size_t)s * act;
  const uint16_t *A2 = a.store + ((size_t)a.n + s) * act;
  const uint16_t *A3 = a.store + ((size_t)2 * a.n + s) * act;
  const uint8_t *cnt = a.counts + s * MM;
  __syncthreads();

  for (int co = 0; co < CH; ++co) {
    const float f = a.feat[s * CH + co];
    const float gz = f > 0.f ? dpred * P[OFF_WL + co] : 0.f;  // d loss / d z4 at the maximum
    if (gz == 0.f) continue;                                   // uniform over the workgroup
    const int Pc = a.argmax[s * CH + co];
    if (Pc < 0 || Pc >= MM) continue;  // only with NaN activations (then gz is not 0)
    for (int i = tid; i < 9 * CH; i += BWD_THREADS) {
      const int q = i / CH, c = i % CH;
      a3w[i] = from_bf16(A3[(size_t)wpos(Pc, q / 3 - 1, q % 3 - 1, M) * CH + c]);
    }
    for (int i = tid; i < 25 * CH; i += BWD_THREADS) {
      const int q = i / CH, c = i % CH;
      a2w[i] = from_bf16(A2[(size_t)wpos(Pc, q / 5 - 2, q % 5 - 2, M) * CH + c]);
    }
    for (int i = tid; i < 49 * CH; i += BWD_THREADS) {
      const int q = i / CH, c = i % CH;
      a1w[i] = from_bf16(A1[(size_t)wpos(Pc, q / 7 - 3, q % 7 - 3, M) * CH + c]);
    }
    for (int i = tid; i < 81; i += BWD_THREADS) xw[i] = (float)cnt[wpos(Pc, i / 9 - 4, i % 9 - 4, M)] * 0.125f;
    __syncthreads();
    // layer 4: weight gradient of channel co and the layer-3 window
    if (tid < 9 * CH) {
      const int d = tid / CH, ci = tid % CH;
      gW4[(co * 9 + d) * CH + ci] += gz * a3w[d * CH + ci];
      dz3[d * CH + ci] = a3w[d * CH + ci] > 0.f ? gz * W4[(co * 9 + d) * CH + ci] : 0.f;
    }
    if (tid == 0) gB4[co] += gz;
    __syncthreads();
    // layer 3: weights from dz3 (3x3) and a2 (5x5); dz2 on the 5x5 window
    for (int e = tid; e < 2304; e += BWD_THREADS) {
      const int c = e / 144, d = (e / CH) % 9, ci = e % CH;
      const int dy = d / 3 - 1, dx = d % 3 - 1;
      float acc = 0.f;
      for (int q = 0; q < 9; ++q) {
        const int qy = q / 3 - 1, qx = q % 3 - 1;
        acc = fmaf(dz3[q * CH + c], a2w[((qy + dy + 2) * 5 + (qx + dx + 2)) * CH + ci], acc);
      }
      gW3[e] += acc;
    }
    if (tid < CH) {
      float acc = 0.f;
      for (int q = 0; q < 9; ++q) acc += dz3[q * CH + tid];
      gB3[tid] += acc;
    }
    for (int e = tid; e < 25 * CH; e += BWD_THREADS) {
      const int r = e / CH, ci = e % CH;
      const int ry = r / 5 - 2, rx = r % 5 - 2;
      float acc = 0.f;
      for (int d = 0; d < 9; ++d) {
        const int qy = ry - (d / 3 - 1), qx = rx - (d % 3 - 1);
        if (qy < -1 || qy > 1 || qx < -1 || qx > 1) continue;
        const int q = (qy + 1) * 3 + (qx + 1);
        for (int c = 0; c < CH; ++c) acc = fmaf(dz3[q * CH + c], W3[(c * 9 + d) * CH + ci], acc);
      }
      dz2[e] = a2w[e] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    // layer 2: weights from dz2 (5x5) and a1 (7x7); dz1 on the 7x7 window
    for (int e = tid; e < 2304; e += BWD_THREADS) {
      const int c = e / 144, d = (e / CH) % 9, ci = e % CH;
      const int dy = d / 3 - 1, dx = d % 3 - 1;
      float acc = 0.f;
      for (int r = 0; r < 25; ++r) {
        const int ry = r / 5 - 2, rx = r % 5 - 2;
        acc = fmaf(dz2[r * CH + c], a1w[((ry + dy + 3) * 7 + (rx + dx + 3)) * CH + ci], acc);
      }
      gW2[e] += acc;
    }
    if (tid < CH) {
      float acc = 0.f;
      for (int r = 0; r < 25; ++r) acc += dz2[r * CH + tid];
      gB2[tid] += acc;
    }
    for (int e = tid; e < 49 * CH; e += BWD_THREADS) {
      const int u = e / CH, ci = e % CH;
      const int uy = u / 7 - 3, ux = u % 7 - 3;
      float acc = 0.f;
      for (int d = 0; d < 9; ++d) {
        const int ry = uy - (d / 3 - 1), rx = ux - (d % 3 - 1);
        if (ry < -2 || ry > 2 || rx < -2 || rx > 2) continue;
        const int r = (ry + 2) * 5 + (rx + 2);
        for (int c = 0; c < CH; ++c) acc = fmaf(dz2[r * CH + c], W2[(c * 9 + d) * CH + ci], acc);
      }
      dz1[e] = a1w[e] > 0.f ? acc : 0.f;
    }
    __syncthreads();
    // layer 1: weights from dz1 (7x7) and the input (9x9)
    if (tid < 144) {
      const int c = tid / 9, d = tid % 9;
      const int dy = d / 3 - 1, dx = d % 3 - 1;
      float acc = 0.f;
      for (int u = 0; u < 49; ++u) {
        const int uy = u / 7 - 3, ux = u % 7 - 3;
        acc = fmaf(dz1[u * CH + c], xw[(uy + dy + 4) * 9 + (ux + dx + 4)], acc);
      }
      gW1[tid] += acc;
    }
    if (tid < CH) {
      float acc = 0.f;
      for (int u = 0; u < 49; ++u) acc += dz1[u * CH + tid];
      gB1[tid] += acc;
    }
    __syncthreads();
  }
  float *out = a.part + s * NPARAM;
  for (int i = tid; i < 2304; i += BWD_THREADS) {
    out[OFF_W2 + i] = gW2[i];
    out[OFF_W3 + i] = gW3[i];
    out[OFF_W4 + i] = gW4[i];
  }
  if (tid < 144) out[OFF_W1 + tid] = gW1[tid];
  if (tid < CH) {
    out[OFF_B1 + tid] = gB1[tid];
    out[OFF_B2 + tid] = gB2[tid];
    out[OFF_B3 + tid] = gB3[tid];
    out[OFF_B4 + tid] = gB4[tid];
    out[OFF_WL + tid] = dpred * a.feat[s * CH + tid];
  }
  if (tid == 0) out[OFF_BL] = dpred;
}

// grad[j] = sum over samples of part[s][j] in a fixed order: chunks of
// RED_CHUNK samples in order (k_cnn_reduce_chunks, one thread per (chunk,
// j)), then the chunk sums in order (k_cnn_reduce).
constexpr int RED_CHUNK = 16;
__global__ void k_cnn_reduce_chunks(const float *part, int64_t n, float *chunks) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (j >= NPARAM) return;
  const int64_t s1 = min(n, (c + 1) * RED_CHUNK);
  float acc = 0.f;
  for (int64_t s = c * RED_CHUNK; s < s1; ++s) acc += part[s * NPARAM + j];
  chunks[c * NPARAM + j] = acc;
}
__global__ void k_cnn_reduce(const float *chunks, int64_t nchunks, float *grad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NPARAM) return;
  float acc = 0.f;
  for (int64_t c = 0; c < nchunks; ++c) acc += chunks[c * NPARAM + j];
  grad[j] = acc;
}

__global__ void k_cnn_loss(const float *pred, const float *target, int64_t n, float *loss) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float d = pred[i] - target[i];
    acc = fmaf(d, d, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

__global__ void k_cnn_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NPARAM) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.f - b1) * gj;
  const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  p[j] -= lr * (mj * c1) / (sqrtf(vj * c2) + eps);
}

struct InitBounds {
  double b[5];  // W1, W2, W3, W4, head
};

__global__ void k_cnn_init(float *p, uint32_t k0, uint32_t k1, InitBounds ib) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NPARAM) return;
  double bound = 0.0;
  if (j < OFF_B1) bound = ib.b[0];
  else if (j >= OFF_W2 && j < OFF_B2) bound = ib.b[1];
  else if (j >= OFF_W3 && j < OFF_B3) bound = ib.b[2];
  else if (j >= OFF_W4 && j < OFF_B4) bound = ib.b[3];
  else if (j >= OFF_WL && j < OFF_BL) bound = ib.b[4];
  float w = 0.f;
  if (bound > 0.0) {
    const Words4 r = philox4x32_10((uint32_t)j, k0, k1, INIT_TAG);
    const double u = ((double)r.w0 + 0.5) / 4294967296.0;
    w = (float)((2.0 * u - 1.0) * bound);
  }
  p[j] = w;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t wrap_lds(int M, int threads) {
  const size_t SS = (size_t)(M + 2) * (M + 2);
  return ((SS + 7) & ~(size_t)7) * 2 + 2 * SS * CH * 2 + (size_t)(threads / 64) * CH * 8;
}
size_t fwd32_lds() {  // A, B [32][33][16] bfloat16, per-wave pooling results
  return (size_t)2 * BUF32 * 2 + (size_t)(THREADS_WRAP / 64) * CH * 8;
}

// Workspace of the training step: stored activations, feat, argmax, pred,
// per-sample gradients.
struct BwdLayout {
  uint16_t *store;
  float *feat, *pred, *part, *chunks;
  int32_t *argmax;
  void *fwd_ws;
  size_t bytes;
};
BwdLayout bwd_layout(int M, int64_t n, void *base) {
  BwdLayout l;
  size_t off = 0;
  auto take = [&](size_t b) {
    void *p = base ? (void *)((char *)base + off) : nullptr;
    off += align256(b);
    return p;
  };
  l.store = (uint16_t *)take((size_t)3 * n * M * M * CH * 2);
  l.feat = (float *)take((size_t)n * CH * 4);
  l.argmax = (int32_t *)take((size_t)n * CH * 4);
  l.pred = (float *)take((size_t)n * 4);
  l.part = (float *)take((size_t)n * NPARAM * 4);
  l.chunks = (float *)take((size_t)((n + RED_CHUNK - 1) / RED_CHUNK) * NPARAM * 4);
  l.fwd_ws = take(cnn_forward_ws(M, n));
  l.bytes = off;
  return l;
}

int check_map(int M, int64_t n) {
  if (M < 2 || M > 2048) return fail_with(MPD_ERR_L, "map size M=%d outside [2, 2048]", M);
  if (n < 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "batch size %lld out of range", (long long)n);
  return MPD_OK;
}

}  // namespace

// Forward workspace: packed weights, then (maps wider than 32) the pooled maxima.
size_t cnn_forward_ws(int M, int64_t n) {
  return align256(PREP_UINT4 * sizeof(uint4)) +
         (M <= WRAP_MAX ? 0 : align256((size_t)n * CH * sizeof(unsigned long long)));
}

int cnn_forward_run(const uint8_t *counts, int M, int64_t n, const float *params, float *pred, float *feat,
                    int32_t *argmax, uint16_t *store, void *ws, hipStream_t stream) {
  if (n == 0) return MPD_OK;
  FwdArgs a;
  a.counts = counts;
  a.M = M;
  a.ntile = (M + TILE - 1) / TILE;
  a.params = params;
  a.pred = pred;
  a.feat = feat;
  a.argmax = argmax;
  a.store = store;
  a.pool = nullptr;
  a.n = n;
  uint4 *Aop = (uint4 *)ws;
  a.Aop = Aop;
  hipLaunchKernelGGL(k_cnn_prep, dim3((PREP_UINT4 + 255) / 256), dim3(256), 0, stream, params, Aop);
  HIP_TRY(hipGetLastError());
  ProfScope ps("k_cnn_forward", stream);
  if (M <= WRAP_MAX) {
    // two workgroups per CU fit in LDS; each walks its share of the maps
    const unsigned grid = (unsigned)std::min<int64_t>(n, 2 * (int64_t)cu_count());
    if (M == 32)
      hipLaunchKernelGGL(k_cnn_forward32, dim3(grid), dim3(THREADS_WRAP), fwd32_lds(), stream, a);
    else
      hipLaunchKernelGGL(k_cnn_forward_wrap<0>, dim3(grid), dim3(THREADS_WRAP), wrap_lds(M, THREADS_WRAP), stream, a);
    HIP_TRY(hipGetLastError());
    return MPD_OK;
  }
  if (store != nullptr) return fail_with(MPD_ERR_L, "stored activations need M <= %d", WRAP_MAX);
  a.pool = (unsigned long long *)((char *)ws + align256(PREP_UINT4 * sizeof(uint4)));
  const int64_t cnt = n * CH;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, a.pool, cnt);
  HIP_TRY(hipGetLastError());
  const unsigned tgrid = (unsigned)std::min<int64_t>(n * a.ntile * a.ntile, cu_count());
  hipLaunchKernelGGL(k_cnn_forward_rtile, dim3(tgrid), dim3(RT_NW * 64), rtile_lds(), stream, a);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_cnn_head, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, a);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

}  // namespace mpd

using namespace mpd;

extern "C" {

int mpd_cnn_init(float *d_params, uint64_t seed, void *stream) {
  g_last_error.clear();
  if (d_params == nullptr || ((uintptr_t)d_params & 3u)) return fail_with(MPD_ERR_PTR, "params NULL or misaligned");
  InitBounds ib;
  const int fan[5] = {9, 144, 144, 144, 16};
  for (int i = 0; i < 5; ++i) ib.b[i] = sqrt(6.0 / fan[i]);
  hipLaunchKernelGGL(k_cnn_init, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_params,
                     (uint32_t)seed, (uint32_t)(seed >> 32), ib);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

size_t mpd_cnn_forward_workspace_bytes(int M, int64_t n) { return n > 0 ? cnn_forward_ws(M, n) : 0; }

int mpd_cnn_forward(const uint8_t *d_counts, int M, int64_t n, const float *d_params, float *d_pred, float *d_feat,
                    int32_t *d_argmax, void *d_workspace, size_t ws_bytes, void *stream) {
  g_last_error.clear();
  int rc = check_map(M, n);
  if (rc != MPD_OK) return rc;
  if (n == 0) return MPD_OK;
  if (d_counts == nullptr || d_params == nullptr || d_pred == nullptr) return fail_with(MPD_ERR_PTR, "NULL argument");
  if (((uintptr_t)d_params | (uintptr_t)d_pred | (uintptr_t)d_feat | (uintptr_t)d_argmax) & 3u)
    return fail_with(MPD_ERR_PTR, "float/int arrays must be 4-byte aligned");
  const size_t need = cnn_forward_ws(M, n);
  if (d_workspace == nullptr || ws_bytes < need)
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
  if ((uintptr_t)d_workspace & 255u) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  return cnn_forward_run(d_counts, M, n, d_params, d_pred, d_feat, d_argmax, nullptr, d_workspace,
                         (hipStream_t)stream);
}

size_t mpd_cnn_train_workspace_bytes(int M, int64_t n) {
  if (M < 2 || M > WRAP_MAX || n <= 0) return 0;
  return bwd_layout(M, n, nullptr).bytes;
}

int mpd_cnn_loss_grad(const uint8_t *d_counts, int M, int64_t n, const float *d_params, const float *d_target,
                      float *d_grad, float *d_loss, float *d_pred, void *d_workspace, size_t ws_bytes,
                      void *stream) {
  g_last_error.clear();
  if (M < 2 || M > WRAP_MAX) return fail_with(MPD_ERR_L, "training needs 2 <= M <= %d (got %d)", WRAP_MAX, M);
  if (n <= 0 || n > (int64_t)1 << 31) return fail_with(MPD_ERR_N, "batch size %lld out of range", (long long)n);
  if (d_counts == nullptr || d_params == nullptr || d_target == nullptr || d_grad == nullptr || d_loss == nullptr)
    return fail_with(MPD_ERR_PTR, "NULL argument");
  if (((uintptr_t)d_params | (uintptr_t)d_target | (uintptr_t)d_grad | (uintptr_t)d_loss | (uintptr_t)d_pred) & 3u)
    return fail_with(MPD_ERR_PTR, "float arrays must be 4-byte aligned");
  const BwdLayout l = bwd_layout(M, n, d_workspace);
  if (d_workspace == nullptr || ws_bytes < l.bytes)
    return fail_with(MPD_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, l.bytes);
  if ((uintptr_t)d_workspace & 255u) return fail_with(MPD_ERR_PTR, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  int rc = cnn_forward_run(d_counts, M, n, d_params, l.pred, l.feat, l.argmax, l.store, l.fwd_ws, st);
  if (rc != MPD_OK) return rc;
  BwdArgs b;
  b.counts = d_counts;
  b.M = M;
  b.n = n;
  b.params = d_params;
  b.store = l.store;
  b.feat = l.feat;
  b.argmax = l.argmax;
  b.pred = l.pred;
  b.target = d_target;
  b.part = l.part;
  {
    ProfScope ps("k_cnn_backward", st);
    hipLaunchKernelGGL(k_cnn_backward, dim3((unsigned)n), dim3(BWD_THREADS), 0, st, b);
  }
  HIP_TRY(hipGetLastError());
  const int64_t nch = (n + RED_CHUNK - 1) / RED_CHUNK;
  hipLaunchKernelGGL(k_cnn_reduce_chunks, dim3((NPARAM + 255) / 256, (unsigned)nch), dim3(256), 0, st, l.part, n,
                     l.chunks);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_cnn_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, st, l.chunks, nch, d_grad);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_cnn_loss, dim3(1), dim3(256), 0, st, l.pred, d_target, n, d_loss);
  HIP_TRY(hipGetLastError());
  if (d_pred != nullptr) HIP_TRY(hipMemcpyAsync(d_pred, l.pred, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  return MPD_OK;
}

int mpd_cnn_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, int step, float lr, float beta1,
                      float beta2, float eps, void *stream) {
  g_last_error.clear();
  if (d_params == nullptr || d_grad == nullptr || d_m == nullptr || d_v == nullptr)
    return fail_with(MPD_ERR_PTR, "NULL argument");
  if (step < 1) return fail_with(MPD_ERR_N, "step counts from 1 (got %d)", step);
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail_with(MPD_ERR_P, "Adam hyper-parameters out of range");
  const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, step)));
  hipLaunchKernelGGL(k_cnn_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_params, d_grad,
                     d_m, d_v, lr, beta1, beta2, eps, c1, c2);
  HIP_TRY(hipGetLastError());
  return MPD_OK;
}

}  // extern "C"
