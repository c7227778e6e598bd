// gfx950 kernels of the neural radiance cache: input encoding, the fused
// BF16 MFMA network (forward, backward, training step) and query resolution.
//
// Network: 80 inputs -> 64 -> 64 -> 64 -> 64 -> 3, ReLU, no biases, weights
// row-major [out][in] in one float array (FP32 master copy; kernels round to
// BF16 when staging them in LDS).  Activations are BF16, products accumulate
// in FP32 (v_mfma_f32_16x16x16_bf16).
//
// Register layout.  A wave works on tiles of 16 samples.  Weights are the A
// operand (rows = output neurons, 16 per tile), samples the N dimension: lane
// i holds A[i%16][4(i/16)+j], B[4(i/16)+j][i%16] and D[4(i/16)+j][i%16].  The
// D tile of output neurons 16t..16t+15 is therefore exactly the B operand of
// the next layer's k-step t, so activations never leave registers in the
// forward pass; the encoding is computed directly into the B chunks of the
// first layer (lane group g = i/16 computes inputs 16s + 4g .. 16s + 4g + 3).
//
// Encoding (80 inputs): a 16-level hash grid over the position normalised to
// the scene box (2 FP16 features per entry, trilinear, dense indexing while
// a level fits the table, else the Instant-NGP spatial hash), 16 real
// spherical harmonics (bands 0-3) of the direction and of the normal, the
// roughness and the albedo, zero padding.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "drt_internal.h"

namespace drt {

#define DEV __device__ __forceinline__

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kW0 = 0, kW1 = 64 * 80, kW2 = kW1 + 4096, kW3 = kW2 + 4096, kW4 = kW3 + 4096;
constexpr int kW4Pad = 16 * 64;             // output layer padded to 16 rows in LDS
constexpr int kLdsW = kW4 + kW4Pad;         // bf16 weights staged in LDS
constexpr int kBlockN = 256;                // 4 waves per workgroup

DEV uint16_t f2bf(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7F800000u) != 0x7F800000u) b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
DEV float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
DEV bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = (short)f2bf(a);
  r[1] = (short)f2bf(b);
  r[2] = (short)f2bf(c);
  r[3] = (short)f2bf(d);
  return r;
}
DEV bf16x4 relu_pack(f32x4 v) {
  return pack4(fmaxf(v[0], 0.f), fmaxf(v[1], 0.f), fmaxf(v[2], 0.f), fmaxf(v[3], 0.f));
}
DEV f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
DEV f32x4 zero4() {
  f32x4 z = {0.f, 0.f, 0.f, 0.f};
  return z;
}
DEV bf16x4 zero_b() {
  bf16x4 z = {0, 0, 0, 0};
  return z;
}

// ---------------------------------------------------------------------------
// weights in LDS, in MFMA fragment order: each 16x16 tile (t, s) of a layer
// (rows 16t.., cols 16s..) is 256 contiguous bf16 laid out as the A operand
// is held -- lane r + 16g owns row 16t + r, cols 16s + 4g .. +3 -- so an A
// load is one contiguous 8-byte read per lane (no bank conflicts).  Layer 4
// is padded to 16 rows (rows 3..15 zero).
// ---------------------------------------------------------------------------
DEV int frag_index(int row, int col, int K) {
  const int t = row >> 4, r = row & 15, s = col >> 4, g = (col >> 2) & 3, j = col & 3;
  return ((t * (K >> 4) + s) << 8) + ((r + 16 * g) << 2) + j;
}

DEV void stage_weights(uint16_t* wl, const float* __restrict__ W) {
  for (int i = threadIdx.x; i < kLdsW; i += blockDim.x) {
    int base, K;
    if (i < kW1) { base = kW0; K = 80; }
    else if (i < kW2) { base = kW1; K = 64; }
    else if (i < kW3) { base = kW2; K = 64; }
    else if (i < kW4) { base = kW3; K = 64; }
    else { base = kW4; K = 64; }
    const int e = i - base, tile = e >> 8, ln = (e & 255) >> 2, j = e & 3;
    const int row = 16 * (tile / (K >> 4)) + (ln & 15);
    const int col = 16 * (tile % (K >> 4)) + 4 * (ln >> 4) + j;
    const float v = (base == kW4 && row >= 3) ? 0.f : W[base + row * K + col];
    wl[i] = f2bf(v);
  }
}
// A operand of W (rows 16t.., cols 16s..)
DEV bf16x4 ldA(const uint16_t* w, int K, int t, int s, int lane) {
  return *reinterpret_cast<const bf16x4*>(w + ((t * (K >> 4) + s) << 8) + 4 * lane);
}
// A operand of W^T (rows = inputs 16t.., k = outputs 16s..): lane r + 16g
// needs W[16s + 4g + j][16t + r], j = 0..3
DEV bf16x4 ldAT(const uint16_t* w, int K, int t, int s, int lane) {
  const int r = lane & 15, g = lane >> 4;
  const uint16_t* p = w + ((s * (K >> 4) + t) << 8) + ((4 * g + 16 * (r >> 2)) << 2) + (r & 3);
  bf16x4 v;
  v[0] = (short)p[0];
  v[1] = (short)p[4];
  v[2] = (short)p[8];
  v[3] = (short)p[12];
  return v;
}

// ---------------------------------------------------------------------------
// encoding
// ---------------------------------------------------------------------------
struct GridLds {
  int res[16];
  int dense[16];
};

DEV void sh16_sel(float x, float y, float z, int g, float o[4]) {
  const float c0 = 0.28209479177387814f, c1 = 0.4886025119029199f;
  const float c2a = 1.0925484305920792f, c2b = 0.31539156525252005f, c2c = 0.5462742152960396f;
  const float c3a = 0.5900435899266435f, c3b = 2.890611442640554f, c3c = 0.4570457994644658f;
  const float c3d = 0.3731763325901154f, c3e = 1.445305721320277f;
  float v[16];
  v[0] = c0;
  v[1] = c1 * y;
  v[2] = c1 * z;
  v[3] = c1 * x;
  v[4] = c2a * x * y;
  v[5] = c2a * y * z;
  v[6] = c2b * (3.f * z * z - 1.f);
  v[7] = c2a * x * z;
  v[8] = c2c * (x * x - y * y);
  v[9] = c3a * y * (3.f * x * x - y * y);
  v[10] = c3b * x * y * z;
  v[11] = c3c * y * (5.f * z * z - 1.f);
  v[12] = c3d * z * (5.f * z * z - 3.f);
  v[13] = c3c * x * (5.f * z * z - 1.f);
  v[14] = c3e * z * (x * x - y * y);
  v[15] = c3a * x * (x * x - 3.f * y * y);
#pragma unroll
  for (int j = 0; j < 4; ++j)
    o[j] = g == 0 ? v[j] : (g == 1 ? v[4 + j] : (g == 2 ? v[8 + j] : v[12 + j]));
}

// Cell of one level: lowest corner c0 and the position's fractions in the cell.
DEV void level_cell(const GridLds& gl, int l, const float xn[3], int c0[3], float fr[3]) {
  const int N = gl.res[l];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float pos = xn[a] * (float)N;
    int c = (int)floorf(pos);
    c = min(max(c, 0), N - 1);
    c0[a] = c;
    fr[a] = pos - (float)c;
  }
}
// Entry of corner k (bit 0: +x, bit 1: +y, bit 2: +z) of the cell: dense
// index while the level fits the table, else the spatial hash -- both
// computed and one selected, so lanes on dense and on hashed levels take
// no divergent branch.
DEV uint32_t corner_entry(const DNrcNet& net, const GridLds& gl, int l, const int c0[3], int k) {
  const uint32_t n1 = (uint32_t)(gl.res[l] + 1);
  const uint32_t mask = (1u << net.log2_table) - 1u;
  const uint32_t cx = c0[0] + (k & 1), cy = c0[1] + ((k >> 1) & 1), cz = c0[2] + ((k >> 2) & 1);
  const uint32_t dense = cx + cy * n1 + cz * n1 * n1;
  const uint32_t hashed = (cx ^ (cy * 2654435761u) ^ (cz * 805459861u)) & mask;
  return gl.dense[l] ? dense : hashed;
}
// Trilinear weight of corner k.
DEV float corner_weight(const float fr[3], int k) {
  return ((k & 1) ? fr[0] : 1.f - fr[0]) * (((k >> 1) & 1) ? fr[1] : 1.f - fr[1]) *
         (((k >> 2) & 1) ? fr[2] : 1.f - fr[2]);
}

// Trilinear corners of one level: index (entry of 2 features) and weight.
DEV void level_corners(const DNrcNet& net, const GridLds& gl, int l, const float xn[3],
                       uint32_t idx[8], float w[8]) {
  int c0[3];
  float fr[3];
  level_cell(gl, l, xn, c0, fr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    w[k] = corner_weight(fr, k);
    idx[k] = corner_entry(net, gl, l, c0, k);
  }
}

DEV void normalise(const DNrcNet& net, const float* rec, float xn[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) xn[a] = fminf(fmaxf((rec[a] - net.lo[a]) * net.inv_ext[a], 0.f), 1.f);
}

// The 20 inputs of lane group g of a sample (B chunks s = 0..4), FP32.
// Chunk 0: hash features 4g..4g+3 = levels 2g, 2g+1; chunk 1: levels 8+2g,
// 9+2g.  The record (64 B, 16-byte aligned) is read whole, and the 32 corner
// entries of the lane's four levels are all requested before any of them
// is used: one memory round trip for the record and one for the grid.
struct Rec {
  float4 a, b, c, d;  // record floats 0..3, 4..7, 8..11, 12..15
};
DEV Rec load_rec(const float* rec) {
  const float4* r4 = reinterpret_cast<const float4*>(rec);
  return Rec{r4[0], r4[1], r4[2], r4[3]};
}

// (An invalid lane -- past the last record -- encodes whatever record it
// holds and gets zeros, selected at the end rather than branched around.)
DEV void encode_rec(const DNrcNet& net, const GridLds& gl, const Rec& R, bool valid, int g,
                    float in[5][4]) {
  const float4 ra = R.a, rb = R.b, rc = R.c, rd = R.d;
  const float p[3] = {ra.x, ra.y, ra.z};
  float xn[3];
  normalise(net, p, xn);
  const int lv[4] = {2 * g, 2 * g + 1, 8 + 2 * g, 9 + 2 * g};
  uint32_t e[4][8];
  float fr[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int c0[3];
    level_cell(gl, lv[q], xn, c0, fr[q]);
    const uint32_t* tab = net.grid + ((size_t)lv[q] << net.log2_table);
#pragma unroll
    for (int k = 0; k < 8; ++k) e[q][k] = tab[corner_entry(net, gl, lv[q], c0, k)];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float f0 = 0.f, f1 = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float w = corner_weight(fr[q], k);
      f0 += w * __half2float(__ushort_as_half((unsigned short)(e[q][k] & 0xFFFFu)));
      f1 += w * __half2float(__ushort_as_half((unsigned short)(e[q][k] >> 16)));
    }
    in[q >> 1][2 * (q & 1)] = f0;
    in[q >> 1][2 * (q & 1) + 1] = f1;
  }
  // record: p 0..2, w_o 3..5, n 6..8, roughness 9, albedo 10..12
  sh16_sel(ra.w, rb.x, rb.y, g, in[2]);
  sh16_sel(rb.z, rb.w, rc.x, g, in[3]);
  in[4][0] = g == 0 ? rc.y : 0.f;
  in[4][1] = g == 0 ? rc.z : 0.f;
  in[4][2] = g == 0 ? rc.w : 0.f;
  in[4][3] = g == 0 ? rd.x : 0.f;
#pragma unroll
  for (int s = 0; s < 5; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) in[s][j] = valid ? in[s][j] : 0.f;
}
// rec must point at a readable record also for an invalid lane
DEV void encode_lane(const DNrcNet& net, const GridLds& gl, const float* rec, bool valid, int g,
                     float in[5][4]) {
  encode_rec(net, gl, load_rec(rec), valid, g, in);
}

DEV void load_grid_tables(GridLds& gl, const DNrcNet& net) {
  if (threadIdx.x < 16) {
    gl.res[threadIdx.x] = net.res[threadIdx.x];
    gl.dense[threadIdx.x] = net.dense[threadIdx.x];
  }
}

// ---------------------------------------------------------------------------
// network forward for one 16-sample tile
// ---------------------------------------------------------------------------
struct Acts {
  bf16x4 h0[5], h1[4], h2[4], h3[4], h4[4];
};

DEV void hidden_layer(const uint16_t* w, int K, const bf16x4* in, int ksteps, bf16x4* out, int lane) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = zero4();
    for (int s = 0; s < ksteps; ++s) acc = mfma(ldA(w, K, t, s, lane), in[s], acc);
    out[t] = relu_pack(acc);
  }
}

// Y: lane group 0 holds the 3 outputs of its sample in Y[0..2]
DEV f32x4 forward_tile(const uint16_t* wl, Acts& A, int lane) {
  hidden_layer(wl + kW0, 80, A.h0, 5, A.h1, lane);
  hidden_layer(wl + kW1, 64, A.h1, 4, A.h2, lane);
  hidden_layer(wl + kW2, 64, A.h2, 4, A.h3, lane);
  hidden_layer(wl + kW3, 64, A.h3, 4, A.h4, lane);
  f32x4 y = zero4();
#pragma unroll
  for (int s = 0; s < 4; ++s) y = mfma(ldA(wl + kW4, 64, 0, s, lane), A.h4[s], y);
  return y;
}

// ---------------------------------------------------------------------------
// backward helpers
// ---------------------------------------------------------------------------
DEV bf16x4 mask_pack(f32x4 g, bf16x4 h) {
  return pack4(h[0] != 0 ? g[0] : 0.f, h[1] != 0 ? g[1] : 0.f, h[2] != 0 ? g[2] : 0.f,
               h[3] != 0 ? g[3] : 0.f);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// B chunks of a tile from explicit inputs x [n][80] (rounded to BF16)
DEV void load_inputs(const float* __restrict__ x, int64_t n, int64_t sample, int lane, bf16x4 h0[5]) {
  const int g = lane >> 4;
  for (int s = 0; s < 5; ++s) {
    if (sample < n) {
      const float* p = x + sample * 80 + 16 * s + 4 * g;
      h0[s] = pack4(p[0], p[1], p[2], p[3]);
    } else {
      h0[s] = zero_b();
    }
  }
}

// Network only: y = net(x) for explicit inputs.
__global__ __launch_bounds__(kBlockN) void k_nrc_forward(const float* __restrict__ W,
                                                        const float* __restrict__ x, int64_t n,
                                                        float* __restrict__ y) {
  __shared__ uint16_t wl[kLdsW];
  stage_weights(wl, W);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t n_tiles = (n + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * (kBlockN / 64) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (kBlockN / 64);
  for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
    int64_t sample = tile * 16 + (lane & 15);
    Acts A;
    load_inputs(x, n, sample, lane, A.h0);
    f32x4 out = forward_tile(wl, A, lane);
    if ((lane >> 4) == 0 && sample < n) {
      y[3 * sample] = out[0];
      y[3 * sample + 1] = out[1];
      y[3 * sample + 2] = out[2];
    }
  }
}

// Encoding only: records [n][16] -> x [n][80] (FP32, before BF16 rounding).
__global__ __launch_bounds__(kBlockN) void k_nrc_encode(DNrcNet net, const float* __restrict__ rec,
                                                       int64_t n, float* __restrict__ x) {
  __shared__ GridLds gl;
  load_grid_tables(gl, net);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int64_t n_tiles = (n + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * (kBlockN / 64) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (kBlockN / 64);
  for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
    int64_t sample = tile * 16 + (lane & 15);
    bool valid = sample < n;
    float in[5][4];
    encode_lane(net, gl, valid ? rec + sample * NRC_REC : rec, valid, g, in);
    if (valid)
      for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[sample * 80 + 16 * s + 4 * g + j] = in[s][j];
  }
}

// Sort of cache queries by spatial key (four launches).  Pass 1, a counting
// sort by the key's top bits (its 32^3 bin): per-block LDS histograms added
// to hist; one-block exclusive scan of hist; per-block ranges reserved in
// the scanned cursors and filled through LDS atomics with (sub-key, item)
// pairs.  Blocks take the same grid-stride subsets in the first and last of
// these launches.  The 128 KB LDS histogram allows one block per CU, so the
// histogram and scatter blocks have 1024 threads (16 waves) and each thread
// requests kSortUnroll keys before it updates any: the passes are bound by
// the latency of those reads.  After the scatter each cursor holds the end
// of its bin.  Pass 2: each bin's pairs counting-sorted by the sub-key (the
// bin's 16^3 sub-cells) in LDS, one bin per workgroup at a time, into the
// final order -- for sorts of at least kRefineMin items; smaller ones are
// ordered by bin only.  The order among equal keys is arbitrary.
constexpr int kSortBlocks = 256;
constexpr int kSortThreads = 1024;
constexpr int kSortUnroll = 4;
constexpr int kRefineBlocks = 512;
constexpr int kRefineThreads = 1024;
constexpr int64_t kRefineMin = (int64_t)1 << 20;  // items

// What is sorted: cache queries with precomputed keys (qbin, first *count
// of capacity), or training records keyed by their positions (valid ones
// of n, qbin null).
struct BinSrc {
  const uint32_t* qbin;
  const int* count;
  int64_t capacity;
  const float* rec;
  const int* valid;
  float lo[3], inv_ext[3];
};
DEV int64_t bin_n(const BinSrc& b) { return b.count ? min((int64_t)*b.count, b.capacity) : b.capacity; }
DEV bool key_of(const BinSrc& b, int64_t i, uint32_t& key) {
  if (b.qbin) {
    key = b.qbin[i];
    return true;
  }
  if (!b.valid[i]) return false;
  const float* r = b.rec + i * NRC_REC;
  key = query_key(r[0], r[1], r[2], b.lo, b.inv_ext);
  return true;
}

// Items of one block (same in the histogram and the scatter pass): rounds
// of kSortThreads x kSortUnroll consecutive items, the block's rounds
// gridDim.x rounds apart; fn(key, item) per valid item, the keys of a
// thread's kSortUnroll items read before any is used.
template <class F>
DEV void for_block_keys(const BinSrc& src, int64_t n, F fn) {
  constexpr int64_t kRound = (int64_t)kSortThreads * kSortUnroll;
  for (int64_t r = (int64_t)blockIdx.x * kRound; r < n; r += (int64_t)gridDim.x * kRound) {
    uint32_t k[kSortUnroll];
    bool ok[kSortUnroll];
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u) {
      const int64_t i = r + (int64_t)u * kSortThreads + threadIdx.x;
      ok[u] = i < n && key_of(src, i, k[u]);
    }
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u)
      if (ok[u]) fn(k[u], r + (int64_t)u * kSortThreads + threadIdx.x);
  }
}

__global__ __launch_bounds__(kSortThreads) void k_query_hist(BinSrc src, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kQueryBins];
  for (int i = threadIdx.x; i < kQueryBins; i += kSortThreads) h[i] = 0;
  __syncthreads();
  for_block_keys(src, bin_n(src), [&](uint32_t k, int64_t) { atomicAdd(&h[k >> kQuerySubBits], 1u); });
  __syncthreads();
  for (int i = threadIdx.x; i < kQueryBins; i += kSortThreads)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ __launch_bounds__(1024) void k_query_scan(uint32_t* __restrict__ hist) {
  constexpr int kPer = kQueryBins / 1024;   // bins per thread
  static_assert(kPer * 1024 == kQueryBins, "one block of 1024 threads");
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  uint32_t sum = 0;
  for (int k = 0; k < kPer; ++k) sum += hist[kPer * t + k];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;
  for (int k = 0; k < kPer; ++k) {
    const uint32_t a = hist[kPer * t + k];
    hist[kPer * t + k] = run;
    run += a;
  }
}

// PAIRS: pairs[pos] = (sub-key, item) at the item's place in its bin (for
// the second pass); else order[pos] = item (bin order only).
template <bool PAIRS>
__global__ __launch_bounds__(kSortThreads) void k_query_scatter(BinSrc src, uint32_t* __restrict__ cursor,
                                                               uint2* __restrict__ pairs,
                                                               int* __restrict__ order) {
  __shared__ uint32_t h[kQueryBins];
  for (int i = threadIdx.x; i < kQueryBins; i += kSortThreads) h[i] = 0;
  __syncthreads();
  const int64_t n = bin_n(src);
  for_block_keys(src, n, [&](uint32_t k, int64_t) { atomicAdd(&h[k >> kQuerySubBits], 1u); });
  __syncthreads();
  for (int i = threadIdx.x; i < kQueryBins; i += kSortThreads)
    if (h[i]) h[i] = atomicAdd(&cursor[i], h[i]);
  __syncthreads();
  for_block_keys(src, n, [&](uint32_t k, int64_t i) {
    const uint32_t pos = atomicAdd(&h[k >> kQuerySubBits], 1u);
    if (PAIRS)
      pairs[pos] = make_uint2(k & (kQuerySubs - 1), (uint32_t)i);
    else
      order[pos] = (int)i;
  });
}

// The pairs [s, e) of one bin over the block's threads, kSortUnroll reads
// requested before any is used (an out-of-range thread reads pair s).
template <class F>
DEV void for_bin_pairs(const uint2* __restrict__ pairs, uint32_t s, uint32_t e, F fn) {
  for (uint32_t i0 = s + threadIdx.x; i0 < e; i0 += kSortUnroll * kRefineThreads) {
    uint2 p[kSortUnroll];
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u) {
      const uint32_t i = i0 + u * kRefineThreads;
      p[u] = pairs[i < e ? i : s];
    }
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u)
      if (i0 + u * kRefineThreads < e) fn(p[u]);
  }
}

// Pass 2: bin b holds pairs [end[b-1], end[b]) (end[-1] = 0); its items are
// written to order in sub-key order.
__global__ __launch_bounds__(kRefineThreads) void k_query_refine(const uint2* __restrict__ pairs,
                                                                const uint32_t* __restrict__ end,
                                                                int* __restrict__ order) {
  // scan: thread t < kScanThreads owns sub-keys [t kPer, (t + 1) kPer)
  constexpr int kPer = kQuerySubs > kRefineThreads ? kQuerySubs / kRefineThreads : 1;
  constexpr int kScanThreads = kQuerySubs / kPer;
  static_assert(kPer * kScanThreads == kQuerySubs && kScanThreads <= kRefineThreads, "scan layout");
  __shared__ uint32_t h[kQuerySubs];
  __shared__ uint32_t part[kScanThreads];
  const int t = threadIdx.x;
  for (int b = blockIdx.x; b < kQueryBins; b += gridDim.x) {
    const uint32_t s = b ? end[b - 1] : 0u, e = end[b];
    if (s >= e) continue;  // the same for the whole block
    for (int i = t; i < kQuerySubs; i += kRefineThreads) h[i] = 0;
    __syncthreads();
    for_bin_pairs(pairs, s, e, [&](uint2 p) { atomicAdd(&h[p.x], 1u); });
    __syncthreads();
    uint32_t c = 0;
    if (t < kScanThreads)
      for (int k = 0; k < kPer; ++k) c += h[kPer * t + k];
    if (t < kScanThreads) part[t] = c;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const uint32_t v = (t < kScanThreads && t >= off) ? part[t - off] : 0u;
      __syncthreads();
      if (t < kScanThreads) part[t] += v;
      __syncthreads();
    }
    if (t < kScanThreads) {  // exclusive offsets of the thread's sub-keys
      uint32_t run = s + part[t] - c;
      for (int k = 0; k < kPer; ++k) {
        const uint32_t n = h[kPer * t + k];
        h[kPer * t + k] = run;
        run += n;
      }
    }
    __syncthreads();
    for_bin_pairs(pairs, s, e, [&](uint2 p) { order[atomicAdd(&h[p.x], 1u)] = (int)p.y; });
    __syncthreads();
  }
}

// hist: kQueryBins counters; pairs: 8-byte aligned, as many as items.
static hipError_t sort_by_key(const BinSrc& src, uint32_t* hist, uint2* pairs, int* order,
                              hipStream_t st) {
  hipError_t e = launch_zero(hist, kQueryBins, st);
  if (e != hipSuccess) return e;
  // up to kSortBlocks workgroups, each with at least 4096 queries: every
  // workgroup clears and flushes a whole LDS histogram, which a small sort
  // (a training frame's records) should not pay 256 times
  const int64_t want = (src.capacity + 4095) / 4096;
  const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > kSortBlocks ? kSortBlocks : want));
  hipLaunchKernelGGL(k_query_hist, dim3(blocks), dim3(kSortThreads), 0, st, src, hist);
  hipLaunchKernelGGL(k_query_scan, dim3(1), dim3(1024), 0, st, hist);
  if (src.capacity < kRefineMin) {
    // a small sort (a training frame's records) stops at the bins: its few
    // items per bin would not pay for the second pass's per-bin work
    hipLaunchKernelGGL(k_query_scatter<false>, dim3(blocks), dim3(kSortThreads), 0, st, src, hist, pairs,
                       order);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_query_scatter<true>, dim3(blocks), dim3(kSortThreads), 0, st, src, hist, pairs,
                     order);
  hipLaunchKernelGGL(k_query_refine, dim3(kRefineBlocks), dim3(kRefineThreads), 0, st, pairs, hist, order);
  return hipGetLastError();
}

// Tiles of this wave when the workgroups of a grid are dealt round-robin to
// the 8 XCDs: XCD x walks its own contiguous tile range [x per, (x + 1) per),
// so with spatially sorted queries its L2 holds the table entries of one
// region at a time.
struct TileRange {
  int64_t first, end, step;
};
DEV TileRange xcd_tiles(int64_t n_tiles) {
  const int n_x = min(8, (int)gridDim.x);
  const int xcd = blockIdx.x % n_x;
  const int64_t blocks_x = (gridDim.x - 1 - xcd) / n_x + 1;
  const int64_t per = (n_tiles + n_x - 1) / n_x;
  TileRange r;
  r.first = (int64_t)xcd * per + (blockIdx.x / n_x) * (kBlockN / 64) + (threadIdx.x >> 6);
  r.end = min(n_tiles, (int64_t)(xcd + 1) * per);
  r.step = blocks_x * (kBlockN / 64);
  return r;
}

// Cache queries: image[qpix] += beta * max(C(record), 0) * inv_spp, for the
// queries in `order` (spatially sorted; null: in slot order), tiles as in
// xcd_tiles.
__global__ __launch_bounds__(kBlockN) void k_nrc_infer(DNrcNet net, const float* __restrict__ W,
                                                      const float* __restrict__ q,
                                                      const int* __restrict__ qpix,
                                                      const int* __restrict__ order,
                                                      const int* __restrict__ count,
                                                      int64_t capacity, float inv_spp,
                                                      float* __restrict__ image) {
  __shared__ uint16_t wl[kLdsW];
  __shared__ GridLds gl;
  stage_weights(wl, W);
  load_grid_tables(gl, net);
  __syncthreads();
  const int64_t n = min((int64_t)*count, capacity);
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const TileRange tr = xcd_tiles((n + 15) / 16);
  if (tr.first >= tr.end) return;
  // Software pipeline over the wave's tiles: the next tile's query index is
  // requested before this tile's grid gathers and its record before this
  // tile's network, so only the gathers' round trip is exposed per tile.
  // Slot indices are below 2^31 (the host bounds the capacity); an invalid
  // lane reads slot 0 (n >= 1 here) and is masked.  The loads are
  // unconditional so that no wait is placed at them.
  auto slot_of = [&](int64_t tile, bool& valid) -> int {
    const int64_t slot = tile * 16 + (lane & 15);
    valid = tile < tr.end && slot < n;
    return valid ? (int)slot : 0;
  };
  auto query_of = [&](int slot) -> int { return order ? order[slot] : slot; };
  bool valid;
  int qi = query_of(slot_of(tr.first, valid));
  Rec rec = load_rec(q + (int64_t)qi * NRC_REC);
  int pix = qpix[qi];
  for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
    bool valid_n;
    const int qi_n = query_of(slot_of(tile + tr.step, valid_n));
    float in[5][4];
    encode_rec(net, gl, rec, valid, g, in);
    const Rec rec_n = load_rec(q + (int64_t)qi_n * NRC_REC);
    const int pix_n = qpix[qi_n];
    Acts A;
#pragma unroll
    for (int s = 0; s < 5; ++s) A.h0[s] = pack4(in[s][0], in[s][1], in[s][2], in[s][3]);
    f32x4 y = forward_tile(wl, A, lane);
    if (g == 0 && valid) {
      float* px = image + 3 * (size_t)pix;
      float c0 = rec.d.y * fmaxf(y[0], 0.f) * inv_spp;
      float c1 = rec.d.z * fmaxf(y[1], 0.f) * inv_spp;
      float c2 = rec.d.w * fmaxf(y[2], 0.f) * inv_spp;
      if (c0 != 0.f) atomicAdd(px, c0);
      if (c1 != 0.f) atomicAdd(px + 1, c1);
      if (c2 != 0.f) atomicAdd(px + 2, c2);
    }
    valid = valid_n;
    rec = rec_n;
    pix = pix_n;
  }
}

// ---------------------------------------------------------------------------
// training in two phases
// ---------------------------------------------------------------------------
// Phase 1 (k_nrc_train_fb): per 16-record tile, forward, relative-L2 output
// gradient, backward propagation of the deltas (no weight gradient), hash-grid
// gradient atomics, and the tile's operands of the weight gradient written to
// a workspace: 38 chunks of 16 features x 16 samples, each stored as the
// register layout holds it (lane r + 16g: features 4g..4g+3 of sample r, one
// 8-byte store per lane).  Chunk map: h0 0-4, h1 5-8, h2 9-12, h3 13-16,
// h4 17-20 (layer inputs), g1 21-24, g2 25-28, g3 29-32, g4 33-36 (masked
// gradients of the hidden outputs), dy 37 (output gradient, rows 0..2).
// Phase 2 (k_nrc_dw, k_nrc_dw_reduce): dW_l = sum over records of
// delta_l (x) h_l, split over records.
constexpr int kChunks = 38;

// Store one chunk transposed to the operand layout of the weight gradient:
// lane r + 16g of the stored chunk holds feature r, samples 4g..4g+3.  The
// register layout (features 4g..4g+3 of sample r) is turned through a
// 16x16 bf16 block of this wave's LDS.
DEV void put_chunk(bf16x4* ws, uint16_t* tb, int64_t tile, int c, bf16x4 v, int lane) {
  const int r = lane & 15, g = lane >> 4;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 4; ++j) tb[(4 * g + j) * 16 + r] = (uint16_t)v[j];
  __builtin_amdgcn_wave_barrier();
  ws[((size_t)tile * kChunks + c) * 64 + lane] = *reinterpret_cast<const bf16x4*>(tb + r * 16 + 4 * g);
}

// Masked deltas of one tile from the output gradient dyb (B layout): gl is
// the gradient at hidden layer l's output, zero where its ReLU was off.
struct Deltas {
  bf16x4 g1[4], g2[4], g3[4], g4[4];
};
DEV void backprop_deltas(const uint16_t* wl, const Acts& A, bf16x4 dyb, Deltas& D, int lane) {
  bf16x4(&g4)[4] = D.g4;
  bf16x4(&g3)[4] = D.g3;
  bf16x4(&g2)[4] = D.g2;
  bf16x4(&g1)[4] = D.g1;
#pragma unroll
  for (int t = 0; t < 4; ++t) g4[t] = mask_pack(mfma(ldAT(wl + kW4, 64, t, 0, lane), dyb, zero4()), A.h4[t]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = zero4();
    for (int s = 0; s < 4; ++s) acc = mfma(ldAT(wl + kW3, 64, t, s, lane), g4[s], acc);
    g3[t] = mask_pack(acc, A.h3[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = zero4();
    for (int s = 0; s < 4; ++s) acc = mfma(ldAT(wl + kW2, 64, t, s, lane), g3[s], acc);
    g2[t] = mask_pack(acc, A.h2[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = zero4();
    for (int s = 0; s < 4; ++s) acc = mfma(ldAT(wl + kW1, 64, t, s, lane), g2[s], acc);
    g1[t] = mask_pack(acc, A.h1[t]);
  }
}

// Input gradient of layer 0 for inputs 16t .. 16t + 15 (accumulator layout:
// lane r + 16g holds inputs 16t + 4g .. +3 of sample r).
DEV f32x4 input_grad_tile(const uint16_t* wl, const Deltas& D, int t, int lane) {
  f32x4 acc = zero4();
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma(ldAT(wl + kW0, 80, t, s, lane), D.g1[s], acc);
  return acc;
}

// Backward propagation of one tile without the weight gradient: the masked
// deltas of every layer, dx of inputs 0..31, and the weight-gradient
// operands written to the workspace (chunk map above).
DEV void backprop_tile(const uint16_t* wl, uint16_t* tb, bf16x4* ws, int64_t tile, const Acts& A,
                       bf16x4 dyb, f32x4 dx[2], int lane) {
  Deltas D;
  backprop_deltas(wl, A, dyb, D, lane);
  const bf16x4(&g4)[4] = D.g4;
  const bf16x4(&g3)[4] = D.g3;
  const bf16x4(&g2)[4] = D.g2;
  const bf16x4(&g1)[4] = D.g1;
#pragma unroll
  for (int t = 0; t < 2; ++t) dx[t] = input_grad_tile(wl, D, t, lane);
  // operands of the weight gradient
#pragma unroll
  for (int c = 0; c < 5; ++c) put_chunk(ws, tb, tile, c, A.h0[c], lane);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    put_chunk(ws, tb, tile, 5 + c, A.h1[c], lane);
    put_chunk(ws, tb, tile, 9 + c, A.h2[c], lane);
    put_chunk(ws, tb, tile, 13 + c, A.h3[c], lane);
    put_chunk(ws, tb, tile, 17 + c, A.h4[c], lane);
    put_chunk(ws, tb, tile, 21 + c, g1[c], lane);
    put_chunk(ws, tb, tile, 25 + c, g2[c], lane);
    put_chunk(ws, tb, tile, 29 + c, g3[c], lane);
    put_chunk(ws, tb, tile, 33 + c, g4[c], lane);
  }
  put_chunk(ws, tb, tile, 37, dyb, lane);
}

// Records are taken in the spatially sorted order of the valid ones
// (order[0 .. *count)), so a tile's records are close together.
__global__ __launch_bounds__(kBlockN) void k_nrc_train_fb(DNrcNet net, const float* __restrict__ W,
                                                         const float* __restrict__ rec,
                                                         const int* __restrict__ order,
                                                         const int* __restrict__ count, int64_t n,
                                                         bf16x4* __restrict__ ws,
                                                         float* __restrict__ dgrid,
                                                         float* __restrict__ loss) {
  __shared__ uint16_t wl[kLdsW];
  __shared__ uint16_t tbuf[kBlockN / 64][256];
  __shared__ GridLds gl;
  __shared__ float loss_acc;
  stage_weights(wl, W);
  load_grid_tables(gl, net);
  if (threadIdx.x == 0) loss_acc = 0.f;
  __syncthreads();
  uint16_t* tb = tbuf[threadIdx.x >> 6];
  const int64_t n_valid = min((int64_t)*count, n);
  const float inv = n_valid > 0 ? 1.0f / (3.0f * (float)n_valid) : 0.f;
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int64_t n_tiles = (n_valid + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * (kBlockN / 64) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (kBlockN / 64);
  float my_loss = 0.f;
  for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
    int64_t slot = tile * 16 + (lane & 15);
    bool ok = slot < n_valid;
    const float* r = rec + (ok ? (int64_t)order[slot] : 0) * NRC_REC;
    float in[5][4];
    encode_lane(net, gl, r, ok, g, in);
    Acts A;
#pragma unroll
    for (int s = 0; s < 5; ++s) A.h0[s] = pack4(in[s][0], in[s][1], in[s][2], in[s][3]);
    f32x4 y = forward_tile(wl, A, lane);
    f32x4 d = zero4();
    if (g == 0 && ok) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float den = y[c] * y[c] + 0.01f;
        float e = y[c] - r[13 + c];
        my_loss += e * e / den;
        d[c] = 2.0f * e / den * inv;
      }
    }
    const bf16x4 dyb = g == 0 ? pack4(d[0], d[1], d[2], 0.f) : zero_b();
    f32x4 dx[2];
    backprop_tile(wl, tb, ws, tile, A, dyb, dx, lane);
    if (ok) {
      // this lane holds d/d inputs {4g+j} and {16+4g+j}: levels 2g, 2g+1, 8+2g, 9+2g
      float xn[3];
      normalise(net, r, xn);
      const int lv[4] = {2 * g, 2 * g + 1, 8 + 2 * g, 9 + 2 * g};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int l = lv[q];
        const float d0 = dx[q >> 1][2 * (q & 1)], d1 = dx[q >> 1][2 * (q & 1) + 1];
        if (d0 == 0.f && d1 == 0.f) continue;
        uint32_t idx[8];
        float w[8];
        level_corners(net, gl, l, xn, idx, w);
        float* tab = dgrid + ((size_t)l << net.log2_table) * 2;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (w[k] == 0.f) continue;
          atomicAdd(tab + 2 * (size_t)idx[k], w[k] * d0);
          atomicAdd(tab + 2 * (size_t)idx[k] + 1, w[k] * d1);
        }
      }
    }
  }
  if (my_loss != 0.f) atomicAdd(&loss_acc, my_loss * inv);
  __syncthreads();
  if (threadIdx.x == 0 && loss_acc != 0.f) atomicAdd(loss, loss_acc);
}

// Network only (test hook), phase 1 on explicit inputs x [n][80] and output
// gradients dy [n][3]: dx [n][80] (inputs 0..31; others 0) and the weight-
// gradient operands; phase 2 then adds dW as in training.
__global__ __launch_bounds__(kBlockN) void k_nrc_backward(const float* __restrict__ W,
                                                         const float* __restrict__ x,
                                                         const float* __restrict__ dy, int64_t n,
                                                         bf16x4* __restrict__ ws,
                                                         float* __restrict__ dx) {
  __shared__ uint16_t wl[kLdsW];
  __shared__ uint16_t tbuf[kBlockN / 64][256];
  stage_weights(wl, W);
  __syncthreads();
  uint16_t* tb = tbuf[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int64_t n_tiles = (n + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * (kBlockN / 64) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (kBlockN / 64);
  for (int64_t tile = wave; tile < n_tiles; tile += n_waves) {
    int64_t sample = tile * 16 + (lane & 15);
    Acts A;
    load_inputs(x, n, sample, lane, A.h0);
    forward_tile(wl, A, lane);
    const bool ok = g == 0 && sample < n;
    const bf16x4 dyb = ok ? pack4(dy[3 * sample], dy[3 * sample + 1], dy[3 * sample + 2], 0.f) : zero_b();
    f32x4 dxv[2];
    backprop_tile(wl, tb, ws, tile, A, dyb, dxv, lane);
    if (dx && sample < n) {
      for (int t = 0; t < 5; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) dx[sample * 80 + 16 * t + 4 * g + j] = t < 2 ? dxv[t][j] : 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// gradient of the cache term through the network's inputs
// ---------------------------------------------------------------------------
// Per query (key order, tiles as in xcd_tiles): forward pass, output gradient
// dy = dL * beta * [y > 0] with dL = adj[pixel] / spp, the masked deltas back
// to layer 0, and the input gradient of inputs 64..67 (roughness, albedo),
// added to the roughness slot and albedo texel the query's vertex read them
// from.  Roughness sums go through LDS for the first kMaxRoughLds slots (all
// queries of a conductor hit one slot).
__global__ __launch_bounds__(kBlockN) void k_nrc_input_grad(
    DNrcNet net, const float* __restrict__ W, const float* __restrict__ q,
    const int* __restrict__ qsample, const int* __restrict__ qref, const int* __restrict__ order,
    const int* __restrict__ count, int64_t capacity, int spp, float inv_spp,
    const float* __restrict__ adj, DGrads G) {
  __shared__ uint16_t wl[kLdsW];
  __shared__ GridLds gl;
  __shared__ float rough_acc[kMaxRoughLds];
  stage_weights(wl, W);
  load_grid_tables(gl, net);
  if (threadIdx.x < kMaxRoughLds) rough_acc[threadIdx.x] = 0.f;
  __syncthreads();
  const int64_t n = min((int64_t)*count, capacity);
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const TileRange tr = xcd_tiles((n + 15) / 16);
  for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
    const int64_t slot = tile * 16 + (lane & 15);
    const bool valid = slot < n;
    const int64_t qi = valid ? (int64_t)order[slot] : 0;
    const float* rec = q + qi * NRC_REC;
    float in[5][4];
    encode_lane(net, gl, rec, valid, g, in);
    Acts A;
#pragma unroll
    for (int s = 0; s < 5; ++s) A.h0[s] = pack4(in[s][0], in[s][1], in[s][2], in[s][3]);
    const f32x4 y = forward_tile(wl, A, lane);
    f32x4 d = zero4();
    if (g == 0 && valid) {
      const float* a = adj + 3 * (size_t)(qsample[qi] / spp);
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = y[c] > 0.f ? a[c] * inv_spp * rec[13 + c] : 0.f;
    }
    const bf16x4 dyb = g == 0 ? pack4(d[0], d[1], d[2], 0.f) : zero_b();
    Deltas D;
    backprop_deltas(wl, A, dyb, D, lane);
    const f32x4 dx = input_grad_tile(wl, D, 4, lane);  // lane group 0: inputs 64..67
    if (g == 0 && valid) {
      const int texel = qref[2 * qi], ids = qref[2 * qi + 1];
      const int tex = ids & 0xff, rslot = (ids >> 8) - 1;
      if (texel >= 0 && G.tex[tex]) {
        float* t = G.tex[tex] + 3 * (size_t)texel;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (dx[1 + c] != 0.f) atomicAdd(t + c, dx[1 + c]);
      }
      if (rslot >= 0 && G.rough && dx[0] != 0.f) {
        if (rslot < kMaxRoughLds) atomicAdd(&rough_acc[rslot], dx[0]);
        else atomicAdd(G.rough + rslot, dx[0]);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kMaxRoughLds && G.rough && rough_acc[threadIdx.x] != 0.f)
    atomicAdd(G.rough + threadIdx.x, rough_acc[threadIdx.x]);
}

// Phase 2: workgroup b takes record tiles [b T, (b+1) T) and writes its
// partial weight gradient to part[b][17600]; k_nrc_dw_reduce adds the
// partials into dW.  Wave 0 owns layer 0 (20 output tiles), waves 1 and 2
// layers 1 and 2 (16 each), wave 3 layers 3 and 4 (16 + 4); operands come
// straight from the workspace (already in operand layout, one 8-byte load
// per lane) and the sums stay in MFMA accumulators.
constexpr int kDwBlockTiles = 16;

template <int NO, int NI>
DEV void dw_layer(const bf16x4* __restrict__ ws, int64_t t0, int64_t t1, int dc0, int hc0,
                  f32x4 (&acc)[NO][NI], int lane) {
  for (int64_t tile = t0; tile < t1; ++tile) {
    const bf16x4* base = ws + (size_t)tile * kChunks * 64 + lane;
    bf16x4 a[NO], b[NI];
#pragma unroll
    for (int o = 0; o < NO; ++o) a[o] = base[(dc0 + o) * 64];
#pragma unroll
    for (int i = 0; i < NI; ++i) b[i] = base[(hc0 + i) * 64];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int i = 0; i < NI; ++i) acc[o][i] = mfma(a[o], b[i], acc[o][i]);
  }
}

// D[4g + j][r] of output tile (o, i) = dW[16 o + 4g + j][16 i + r]
template <int NO, int NI>
DEV void dw_store(float* __restrict__ part, int base, int K, int rows, const f32x4 (&acc)[NO][NI],
                  int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * o + 4 * g + j;
        if (row < rows) part[base + row * K + 16 * i + r] = acc[o][i][j];
      }
}

template <int NO, int NI>
DEV void dw_job(const bf16x4* ws, int64_t t0, int64_t t1, int dc0, int hc0, float* part, int base,
                int K, int rows, int lane) {
  f32x4 acc[NO][NI];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int i = 0; i < NI; ++i) acc[o][i] = zero4();
  dw_layer<NO, NI>(ws, t0, t1, dc0, hc0, acc, lane);
  dw_store<NO, NI>(part, base, K, rows, acc, lane);
}

__global__ __launch_bounds__(kBlockN) void k_nrc_dw(const bf16x4* __restrict__ ws,
                                                   const int* __restrict__ count, int64_t n,
                                                   float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t n_tiles = ((count ? min((int64_t)*count, n) : n) + 15) / 16;  // tiles phase 1 wrote
  const int64_t t0 = (int64_t)blockIdx.x * kDwBlockTiles;
  const int64_t t1 = min(n_tiles, t0 + kDwBlockTiles);
  float* p = part + (size_t)blockIdx.x * (kW4 + 3 * 64);
  if (wv == 0) {
    dw_job<4, 5>(ws, t0, t1, 21, 0, p, kW0, 80, 64, lane);
  } else if (wv == 1) {
    dw_job<4, 4>(ws, t0, t1, 25, 5, p, kW1, 64, 64, lane);
  } else if (wv == 2) {
    dw_job<4, 4>(ws, t0, t1, 29, 9, p, kW2, 64, 64, lane);
  } else {
    dw_job<4, 4>(ws, t0, t1, 33, 13, p, kW3, 64, 64, lane);
    dw_job<1, 4>(ws, t0, t1, 37, 17, p, kW4, 64, 3, lane);
  }
}

// dW[i] += sum over workgroups b of part[b][i]: workgroup (x, y) sums
// partials 16y .. 16y+15 of weights 256x .. 256x+255 and adds the sum.
constexpr int kReduceSlice = 16;
__global__ __launch_bounds__(kBlockN) void k_nrc_dw_reduce(const float* __restrict__ part, int nb,
                                                          float* __restrict__ dW) {
  const int i = blockIdx.x * kBlockN + threadIdx.x;
  if (i >= kW4 + 3 * 64) return;
  const int b0 = blockIdx.y * kReduceSlice, b1 = min(nb, b0 + kReduceSlice);
  float s = 0.f;
  for (int b = b0; b < b1; ++b) s += part[(size_t)b * (kW4 + 3 * 64) + i];
  if (s != 0.f) atomicAdd(dW + i, s);
}

// Hash-grid gradient only: dgrid += trilinear scatter of dx [n][80] (inputs
// 0..31) at the records' positions.  One lane per (record, level).
__global__ __launch_bounds__(kBlockN) void k_nrc_grid_backward(DNrcNet net,
                                                              const float* __restrict__ rec,
                                                              const float* __restrict__ dx,
                                                              int64_t n, float* __restrict__ dgrid) {
  __shared__ GridLds gl;
  load_grid_tables(gl, net);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlockN + threadIdx.x;
  if (i >= n * 16) return;
  const int64_t r = i / 16;
  const int l = (int)(i % 16);
  const float d0 = dx[r * 80 + 2 * l], d1 = dx[r * 80 + 2 * l + 1];
  if (d0 == 0.f && d1 == 0.f) return;
  float xn[3];
  normalise(net, rec + r * NRC_REC, xn);
  uint32_t idx[8];
  float w[8];
  level_corners(net, gl, l, xn, idx, w);
  float* tab = dgrid + ((size_t)l << net.log2_table) * 2;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (w[k] == 0.f) continue;
    atomicAdd(tab + 2 * (size_t)idx[k], w[k] * d0);
    atomicAdd(tab + 2 * (size_t)idx[k] + 1, w[k] * d1);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_nrc_grid_backward(const DNrcNet& net, const float* rec, const float* dx,
                                    int64_t n, float* dgrid, hipStream_t st) {
  int64_t blocks = (n * 16 + kBlockN - 1) / kBlockN;
  hipLaunchKernelGGL(k_nrc_grid_backward, dim3((unsigned)blocks), dim3(kBlockN), 0, st, net, rec, dx,
                     n, dgrid);
  return hipGetLastError();
}
static unsigned grid_for(int64_t n, int64_t max_blocks) {
  int64_t tiles = (n + 15) / 16;
  int64_t blocks = (tiles + (kBlockN / 64) - 1) / (kBlockN / 64);
  if (blocks < 1) blocks = 1;
  if (blocks > max_blocks) blocks = max_blocks;
  return (unsigned)blocks;
}

hipError_t launch_nrc_forward(const float* W, const float* x, int64_t n, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_nrc_forward, dim3(grid_for(n, 4096)), dim3(kBlockN), 0, st, W, x, n, y);
  return hipGetLastError();
}

hipError_t launch_nrc_encode(const DNrcNet& net, const float* rec, int64_t n, float* x,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_nrc_encode, dim3(grid_for(n, 4096)), dim3(kBlockN), 0, st, net, rec, n, x);
  return hipGetLastError();
}
hipError_t launch_query_sort(const uint32_t* qbin, const int* count, int64_t capacity,
                             uint32_t* hist, void* pairs, int* order, hipStream_t st) {
  BinSrc src = {};
  src.qbin = qbin;
  src.count = count;
  src.capacity = capacity;
  return sort_by_key(src, hist, static_cast<uint2*>(pairs), order, st);
}
hipError_t launch_nrc_infer(const DNrcNet& net, const float* W, const float* q, const int* qpix,
                            const int* order, const int* count, int64_t capacity, float inv_spp,
                            float* image, hipStream_t st) {
  // persistent: 4 workgroups per CU (LDS-limited), each wave loops over tiles
  hipLaunchKernelGGL(k_nrc_infer, dim3(grid_for(capacity, 1024)), dim3(kBlockN), 0, st, net, W, q,
                     qpix, order, count, capacity, inv_spp, image);
  return hipGetLastError();
}
hipError_t launch_nrc_input_grad(const DNrcNet& net, const float* W, const float* q,
                                 const int* qsample, const int* qref, const int* order,
                                 const int* count, int64_t capacity, int spp, const float* adj,
                                 const DGrads& g, hipStream_t st) {
  hipLaunchKernelGGL(k_nrc_input_grad, dim3(grid_for(capacity, 1024)), dim3(kBlockN), 0, st, net,
                     W, q, qsample, qref, order, count, capacity, spp, 1.0f / (float)spp, adj, g);
  return hipGetLastError();
}
// workspace: operand chunks of every record tile | phase-2 partials |
// sort pairs [n] (8 bytes each) | sorted record order [n] | bin histogram
static int64_t dw_blocks(int64_t n) { return ((n + 15) / 16 + kDwBlockTiles - 1) / kDwBlockTiles; }
static int64_t ws_chunk_bytes(int64_t n) { return ((n + 15) / 16) * kChunks * 64 * 8; }
static int64_t ws_part_bytes(int64_t n) { return dw_blocks(n) * (kW4 + 3 * 64) * 4; }
static int64_t ws_pairs_offset(int64_t n) { return (ws_chunk_bytes(n) + ws_part_bytes(n) + 7) & ~(int64_t)7; }
int64_t nrc_train_workspace_bytes(int64_t n) {
  return ws_pairs_offset(n) + n * 8 + n * 4 + kQueryBins * 4;
}

hipError_t launch_nrc_backward(const float* W, const float* x, const float* dy, int64_t n, void* ws,
                               float* dW, float* dx, hipStream_t st) {
  const int64_t n_tiles = (n + 15) / 16;
  if (n_tiles == 0) return hipSuccess;
  float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + ws_chunk_bytes(n));
  hipLaunchKernelGGL(k_nrc_backward, dim3(grid_for(n, 1024)), dim3(kBlockN), 0, st, W, x, dy, n,
                     reinterpret_cast<bf16x4*>(ws), dx);
  const int64_t blocks = dw_blocks(n);
  hipLaunchKernelGGL(k_nrc_dw, dim3((unsigned)blocks), dim3(kBlockN), 0, st,
                     reinterpret_cast<const bf16x4*>(ws), (const int*)nullptr, n, part);
  hipLaunchKernelGGL(k_nrc_dw_reduce,
                     dim3((kW4 + 3 * 64 + kBlockN - 1) / kBlockN,
                          (unsigned)((blocks + kReduceSlice - 1) / kReduceSlice)),
                     dim3(kBlockN), 0, st, part, (int)blocks, dW);
  return hipGetLastError();
}

hipError_t launch_nrc_train(const DNrcNet& net, const float* W, const float* rec, const int* valid,
                             const int* count, int64_t n, void* ws, float* dW, float* dgrid,
                             float* loss, hipStream_t st) {
  const int64_t n_tiles = (n + 15) / 16;
  if (n_tiles == 0) return hipSuccess;
  char* base = static_cast<char*>(ws);
  float* part = reinterpret_cast<float*>(base + ws_chunk_bytes(n));
  uint2* pairs = reinterpret_cast<uint2*>(base + ws_pairs_offset(n));
  int* order = reinterpret_cast<int*>(pairs + n);
  uint32_t* hist = reinterpret_cast<uint32_t*>(order + n);
  BinSrc src = {};
  src.capacity = n;
  src.rec = rec;
  src.valid = valid;
  for (int a = 0; a < 3; ++a) {
    src.lo[a] = net.lo[a];
    src.inv_ext[a] = net.inv_ext[a];
  }
  hipError_t e = sort_by_key(src, hist, pairs, order, st);
  if (e != hipSuccess) return e;
  // 2 workgroups per CU fit in registers; waves loop over tiles
  hipLaunchKernelGGL(k_nrc_train_fb, dim3(grid_for(n, 1024)), dim3(kBlockN), 0, st, net, W, rec,
                     order, count, n, reinterpret_cast<bf16x4*>(ws), dgrid, loss);
  const int64_t blocks = dw_blocks(n);
  hipLaunchKernelGGL(k_nrc_dw, dim3((unsigned)blocks), dim3(kBlockN), 0, st,
                     reinterpret_cast<const bf16x4*>(ws), count, n, part);
  hipLaunchKernelGGL(k_nrc_dw_reduce,
                     dim3((kW4 + 3 * 64 + kBlockN - 1) / kBlockN,
                          (unsigned)((blocks + kReduceSlice - 1) / kReduceSlice)),
                     dim3(kBlockN), 0, st, part, (int)blocks, dW);
  return hipGetLastError();
}

}  // namespace drt
