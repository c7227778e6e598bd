// Internal layout shared by the host runtime (drt_host.cpp) and the gfx950
// kernels (drt_kernels.hip).  Everything here is plain data: the scene lives
// in one caller-owned device buffer, addressed through the pointers of
// DScene, which is passed to every kernel by value.
#pragma once
#include <cstddef>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/drt.h"

namespace drt {

// BVH traversal stack depth (entries per lane, held in LDS).  The binary
// build keeps interior nodes at depth < kMaxInteriorDepth; the four-wide
// nodes are the binary interior nodes at even depth (so at most 12 levels
// of them), and a visit pushes at most 3 children, so the stack never holds
// more than 3 x 12 = 36 = kStackDepth entries.  36 entries x 64 lanes keep
// sixteen one-wave workgroups per CU within the 160 KB of LDS.
constexpr int kStackDepth = 36;
// Small scenes: the megakernels that render (primal, adjoint, cached modes)
// copy the whole tree and its triangles into each workgroup's LDS, beside a
// traversal stack of kStackDepthSmall entries (trees of up to 5 four-wide
// levels), when they fit in kLdsSceneBytes: node and triangle reads then
// come from LDS instead of the L1.  Stack, copy and the kernels' other LDS
// stay within 10 KB per one-wave workgroup, 16 per CU as without the copy.
constexpr int kStackDepthSmall = 16;
constexpr int kLdsSceneBytes = 5120;
constexpr int kMaxInteriorDepth = 24;
constexpr int kBlock = 64;             // threads per workgroup of the megakernels (one wave)
constexpr int kTile = 8;               // workgroup = 8 x 8 pixel tile
// Tiles covering n pixels (n up to INT32_MAX: computed in 64 bits).
__host__ __device__ inline int32_t tiles_of(int32_t n) {
  return (int32_t)(((int64_t)n + kTile - 1) / kTile);
}
// The launch grid's y extent holds the tile rows: images up to 65535 tiles
// (524,280 pixels) high.
constexpr int32_t kMaxTileRows = 65535;
constexpr int kMaxRoughLds = 64;       // roughness slots pre-reduced in LDS
// The replayed adjoint splits each tile's samples over this many workgroups
// (contiguous sample ranges): four times more, shorter waves leave less of
// the GPU idle at the end of the launch.  The launch and the size of the
// intersection records both take the factor from adjoint_split().
constexpr int kAdjointSplit = 4;
__host__ __device__ inline int adjoint_split(int spp) { return spp < kAdjointSplit ? spp : kAdjointSplit; }

// Four-child BVH node, 128 bytes (one L2 line): the children's boxes by
// coordinate (one float4 per bound: lo x, lo y, lo z, hi x, hi y, hi z of the
// four children, so a ray loads the near and the far bound of each axis as
// whole float4 and needs no min / max to order them), then per child an
// interior node index (count 0), a leaf's triangle range (count > 0) or
// nothing (count -1).  An empty slot holds a zero box.
struct alignas(16) DNode {
  float box[6][4];
  int32_t child[4];
  int32_t count[4];
};
static_assert(sizeof(DNode) == 128, "DNode");

// Triangle in BVH leaf order, 48 bytes: vertices, original id, flags.
struct alignas(16) DTri {
  float p0x, p0y, p0z, p1x;
  float p1y, p1z, p2x, p2y;
  float p2z;
  int32_t prim;    // original triangle id
  int32_t flags;   // bit 0: pass-through (null) surface, skipped by shadow rays
  int32_t pad;
};
static_assert(sizeof(DTri) == 48, "DTri");
// the traversal reads vertex v's component c at float 3 v + c, prim at 9, flags at 10
static_assert(offsetof(DTri, p2z) == 8 * sizeof(float) && offsetof(DTri, prim) == 9 * sizeof(float) &&
                  offsetof(DTri, flags) == 10 * sizeof(float),
              "DTri layout");

// Shading attributes by original triangle id, 32 bytes.
struct alignas(16) DShade {
  float u0, v0, u1, v1;
  float u2, v2;
  int32_t material, emitter;
  float nx, ny, nz;  // unit geometric normal, (p1 - p0) x (p2 - p0) normalised
  int32_t pad;
};
static_assert(sizeof(DShade) == 48, "DShade");

struct alignas(16) DMaterial {
  int32_t type, texture, rough_slot, pad;
  float albedo[3], alpha;
  float f0[3], eta;
  float opacity, pad2[3];
};
static_assert(sizeof(DMaterial) == 64, "DMaterial");

struct alignas(16) DEmitter {
  int32_t type, pad0, pad1, pad2;
  float p0[3], area;
  float e1[3], pad3;
  float e2[3], pad4;
  float n[3], pad5;
  float radiance[3], pad6;
};
static_assert(sizeof(DEmitter) == 96, "DEmitter");

struct DScene {
  const DNode* nodes;
  const DTri* tris;
  const DShade* shade;
  const DMaterial* mats;
  const DEmitter* ems;
  const float* env;          // [h][w][3]
  const float* env_puv;      // [h][w]: density in (u, v) of the sampling distribution
  const float* env_cdf_row;  // [h+1]
  const float* env_cdf_col;  // [h][w+1]
  int32_t n_ems, env_w, env_h, env_emitter;
  int32_t n_mats, n_rough, n_tex;
  int32_t lds_scene;         // the tree and triangles fit the megakernels' LDS copy
  int32_t n_nodes, n_tris;
  float eps;
  int32_t tex_w[DRT_MAX_TEXTURES], tex_h[DRT_MAX_TEXTURES];
};

struct DParams {
  const float* tex[DRT_MAX_TEXTURES];
  const float* rough;
};

struct DGrads {
  float* tex[DRT_MAX_TEXTURES];
  float* rough;
};

struct DCam {
  float ox, oy, oz;
  float fx, fy, fz;   // forward
  float rx, ry, rz;   // right
  float ux, uy, uz;   // up
  float tan_half, aspect;
};

struct DCams {
  int32_t n, width, height, pad;
  DCam cam[DRT_MAX_CAMERAS];
};

struct DRender {
  int32_t spp, max_depth, rr_depth;
  uint32_t flags;
  uint32_t key0, key1;
  uint64_t* stats;
  // replayed adjoint: pass A's intersections, [workgroup][max_depth][kBlock]
  // records of (triangle or -1, b1, b2, shadow ray unoccluded), which the
  // replay reads instead of tracing again (null: the replay traces); the
  // cached replay's: [workgroup][spp][max_depth][kBlock]
  int4* hits;
  // replayed adjoint with records: work counter of its persistent workgroups
  // (zeroed before the launch; it lives in the caller's record buffer)
  uint32_t* items;
};

// Radiance-cache record: 16 floats = position[3], direction[3], normal[3],
// roughness, albedo[3], then throughput[3] (queries) or target[3] (training).
constexpr int NRC_REC = 16;

// Radiance-cache network view for the kernels.
struct DNrcNet {
  const uint32_t* grid;  // [16 levels][2^log2_table] entries of 2 FP16 features
  int log2_table;
  int res[16];           // level resolutions
  int dense[16];         // 1 if the level is indexed densely
  float lo[3], inv_ext[3];
};

// Outputs of the cached primal (queries) and of the training paths.
struct DNrcIO {
  float* rec;       // [capacity or n_paths][NRC_REC]
  int* qpix;        // queries: image index of each query
  int* valid;       // training: 1 if path j has a record
  int* count;       // appended queries / valid records
  int64_t capacity; // queries the buffer holds
  int K;            // record vertex index
  float* lsamp;     // per-sample radiance [n_samples][3] (cached adjoint), else null
  uint32_t* qbin;   // queries: spatial key of each query (null: not sorted)
  int* qref;        // queries: [2] per query, the parameters its inputs were read
                    // from (query_ref_put), or null (not recorded)
  float* trec;      // self-training: records [n_paths * (K - 1)][NRC_REC]
  float* tbeta;     // self-training: throughput at each record [n_paths * (K - 1)][3]
  int* rcount;      // self-training: records written
  float lo[3], inv_ext[3];  // scene box of the cache (query binning)
};

// Scene parameters behind a query's inputs, two ints per query: the albedo
// texel (-1: the albedo input is a constant) and texture | (roughness slot +
// 1) << 8 (slot + 1 = 0: the roughness input is a constant).
__host__ __device__ inline void query_ref_put(int* q, int texel, int tex, int rough_slot) {
  q[0] = texel;
  q[1] = (tex & 0xff) | ((rough_slot + 1) << 8);
}

// Spatial key of cache queries: the Morton code (27 bits) of the query's
// cell among 512 cells per axis of the cache's box, so that key-sorted
// queries gather nearby table entries.  The sort takes two passes: a
// counting sort by the top 15 bits (32^3 bins, as many as one workgroup's
// LDS histogram holds), then, for sorts of 2^20 items or more, each bin's
// queries by the low 12 bits (its 16^3 sub-cells).  Inference of 40M queries
// (1024^2, 64 spp) measured by the order's cells: 32^3 12.6 ms, 64^3
// 10.7 ms, 128^3 9.2 ms, 256^3 8.1-8.4 ms, 512^3 7.7 ms, 1024^3 7.2 ms;
// unsorted 26.4 ms.
constexpr int kQueryKeyBits = 9;                                    // per axis
constexpr int kQueryBinBits = 5;                                    // first pass, per axis
constexpr int kQueryBins = 1 << (3 * kQueryBinBits);
constexpr int kQuerySubBits = 3 * (kQueryKeyBits - kQueryBinBits);  // second pass
constexpr int kQuerySubs = 1 << kQuerySubBits;
__host__ __device__ inline uint32_t query_key(float x, float y, float z, const float lo[3],
                                              const float inv_ext[3]) {
  const float v[3] = {x, y, z};
  uint32_t m = 0;
  for (int a = 0; a < 3; ++a) {
    float t = (v[a] - lo[a]) * inv_ext[a] * (float)(1 << kQueryKeyBits);
    int c = (int)t;
    c = c < 0 ? 0 : (c > (1 << kQueryKeyBits) - 1 ? (1 << kQueryKeyBits) - 1 : c);
    for (int b = 0; b < kQueryKeyBits; ++b) m |= (uint32_t)((c >> b) & 1) << (3 * b + a);
  }
  return m;
}

// Launchers (drt_kernels.hip).
hipError_t launch_render_forward(const DScene& s, const DParams& p, const DCams& c,
                                 const DRender& r, float* image, hipStream_t st);
hipError_t launch_render_cached(const DScene& s, const DParams& p, const DCams& c,
                                const DRender& r, float* image, const DNrcIO& io,
                                hipStream_t st);
hipError_t launch_nrc_records(const DScene& s, const DParams& p, const DCams& c, const DRender& r,
                              int64_t n_paths, const DNrcIO& io, hipStream_t st);
// Self-training paths (render_pixel<MODE_TRAIN_SELF>), then, once the
// queries are answered into io.lsamp, the records' targets.
hipError_t launch_nrc_records_self(const DScene& s, const DParams& p, const DCams& c,
                                   const DRender& r, int64_t n_paths, const DNrcIO& io,
                                   hipStream_t st);
hipError_t launch_nrc_self_targets(const DNrcIO& io, int64_t n_paths, hipStream_t st);
hipError_t launch_render_adjoint(const DScene& s, const DParams& p, const DCams& c,
                                 const DRender& r, const float* adj, const DGrads& g,
                                 hipStream_t st);
// Workgroups of the persistent replayed adjoint (with records) on the current
// device: as many as can be resident at once (0 if the device cannot be
// queried).  The launch and the record size both use it.
int adjoint_resident_groups();
// Devices the per-device caches of the library cover.
constexpr int kMaxDevices = 64;
// Scratch of drt_render_adjoint_noalloc: the 256-byte work-counter header
// and 32 MiB of record slots (4096 resident workgroups x depth 8 x 64 lanes
// x 16 B).
constexpr int64_t kNoAllocScratchBytes = DRT_NOALLOC_SCRATCH_BYTES;
// Address of the calling thread's current device's copy of that scratch,
// looked up once per device (hipGetSymbolAddress) and cached.
hipError_t noalloc_scratch(void** out);
hipError_t launch_render_adjoint_cached(const DScene& s, const DParams& p, const DCams& c,
                                        const DRender& r, const float* adj, const DGrads& g,
                                        const DNrcIO& io, hipStream_t st);
hipError_t launch_render_jvp(const DScene& s, const DParams& p, const DCams& c, const DRender& r,
                             const DGrads& t, float* image, hipStream_t st);
int64_t wavefront_workspace_bytes(int64_t n_paths);
int64_t wavefront_adjoint_workspace_bytes(int64_t n_paths);
hipError_t launch_render_adjoint_wavefront(const DScene& s, const DParams& p, const DCams& c,
                                           const DRender& r, const float* adj, const DGrads& G,
                                           void* ws, hipStream_t st);
hipError_t launch_render_wavefront(const DScene& s, const DParams& p, const DCams& c,
                                   const DRender& r, void* ws, float* image, hipStream_t st);
// Checkpointed adjoint (drt_wavefront.hip): forward pass keeping the ray
// state of every bounce, then the backward pass from those checkpoints.
int64_t checkpoint_workspace_bytes(int64_t n_paths, int max_depth);
hipError_t launch_render_checkpoint_forward(const DScene& s, const DParams& p, const DCams& c,
                                            const DRender& r, void* ws, float* image,
                                            hipStream_t st);
hipError_t launch_render_checkpoint_adjoint(const DScene& s, const DParams& p, const DCams& c,
                                            const DRender& r, const float* adj, const DGrads& G,
                                            void* ws, hipStream_t st);
hipError_t launch_trace(const DScene& s, const float* rays, int64_t n, int mode, drt_hit* hits,
                        hipStream_t st);
hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out,
                         hipStream_t st);
int64_t loss_workspace_floats(int64_t n);
hipError_t launch_loss_l2(const float* img, const float* tgt, int64_t n, float* adj, float* loss,
                          float* ws, hipStream_t st);
hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n,
                       const drt_adam_opts& o, hipStream_t st);
hipError_t launch_zero(void* p, int64_t n_words, hipStream_t st);
// Launchers (drt_nrc.hip).
hipError_t launch_nrc_forward(const float* W, const float* x, int64_t n, float* y, hipStream_t st);
hipError_t launch_nrc_backward(const float* W, const float* x, const float* dy, int64_t n, void* ws,
                               float* dW, float* dx, hipStream_t st);
hipError_t launch_nrc_encode(const DNrcNet& net, const float* rec, int64_t n, float* x,
                             hipStream_t st);
// Sort of the queries by spatial key (qbin): order[] = query indices in key
// order (for fewer than 2^20 queries, in bin order).  hist: kQueryBins words
// of scratch; pairs: 8-byte aligned scratch of capacity 8-byte entries.
hipError_t launch_query_sort(const uint32_t* qbin, const int* count, int64_t capacity,
                             uint32_t* hist, void* pairs, int* order, hipStream_t st);
hipError_t launch_nrc_infer(const DNrcNet& net, const float* W, const float* q, const int* qpix,
                            const int* order, const int* count, int64_t capacity, float inv_spp,
                            float* image, hipStream_t st);
// Gradient of the cache term through the network's albedo and roughness
// inputs: queries q with sample ids qsample (pixel = id / spp), references
// qref, in the key order of launch_query_sort; adj: image adjoint.
hipError_t launch_nrc_input_grad(const DNrcNet& net, const float* W, const float* q,
                                 const int* qsample, const int* qref, const int* order,
                                 const int* count, int64_t capacity, int spp, const float* adj,
                                 const DGrads& g, hipStream_t st);
hipError_t launch_nrc_grid_backward(const DNrcNet& net, const float* rec, const float* dx,
                                    int64_t n, float* dgrid, hipStream_t st);
int64_t nrc_train_workspace_bytes(int64_t n);
hipError_t launch_nrc_train(const DNrcNet& net, const float* W, const float* rec, const int* valid,
                             const int* count, int64_t n, void* ws, float* dW, float* dgrid,
                             float* loss, hipStream_t st);

}  // namespace drt
