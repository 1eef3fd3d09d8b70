// fpsz_internal.h -- shared definitions of the gfx950 library (format
// constants, the per-call plan, device parameter block, wave primitives).
//
// Format (little-endian, 8-byte aligned sections):
//   header (256 B) | code_len u8[1036] | tile_word_offset u64[T+1] |
//   tile_exc_offset u64[T+1] | chunk_bits u16[C] | exceptions {u32 key, u32 val}[E] |
//   words u32[W]
// Stream order: tiles row-major over the tile grid, points row-major inside
// the edge-clipped tile.  Tiles: 1D 8192, 2D 64x128, 3D 16x16x32 points.
// Each tile's bits form one MSB-first stream cut into chunks of 128 symbols
// (chunk_bits records each chunk's length) and padded to a 32-bit word.
// Symbol of a Lorenzo residual d: |d| <= 511 -> d + 512; 512 <= |d| < 2^15 ->
// 1024 + 2(k - 9) + (d < 0) followed by k raw bits of |d| - 2^k, k = floor
// log2 |d|; |d| >= 2^15 -> symbol 0 with d in the exception list.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fpsz.h"

namespace fpsz {

constexpr uint32_t kMagic = 0x5A535046u;  // "FPSZ"
constexpr uint16_t kVersion = 1;
constexpr uint64_t kHdr = 256;
constexpr int kNSym = 1036;
constexpr int kLMax = 18;
constexpr int kChunk = 128;
constexpr int kTilePts = 8192;
constexpr int kLutBits = 11;
constexpr uint32_t kTagPatch = 0x80000000u;
constexpr uint16_t kFlagConst = 1, kFlagTile = 2, kFlagClosed = 4, kFlagInloop = 8,
                   kFlagXform = 16;
// Plan::variant: plain Lorenzo on prequantized bins, SZ 1.4-style in-loop
// prediction, or the orthogonal block transform (the last two tile domain)
enum : int32_t { kVarPlain = 0, kVarInloop = 1, kVarXform = 2 };
constexpr int kBlock = 256;
constexpr int kRangeBlocks = 1024;
// The compressor's histogram is kept in this many copies (workgroup b adds
// into copy b % kHistCopies), so that the hot bins of many workgroups do not
// all contend for one address; the codebook kernel sums them into copy 0.
constexpr int kHistCopies = 16;
constexpr int kVerifyBlocks = 1024;

// header byte offsets
enum : uint32_t {
  H_MAGIC = 0, H_VERSION = 4, H_FLAGS = 6, H_DTYPE = 8, H_NDIM = 9, H_LOG2D = 10,
  H_LOG2R = 11, H_LMAX = 12, H_DIMS = 16, H_TILE = 40, H_CHUNK = 52, H_PSNR = 56,
  H_EBREL = 64, H_VR = 72, H_EB = 80, H_E2 = 88, H_R = 96, H_E2T = 104, H_RT = 112,
  H_MIN = 120, H_MAX = 128, H_N = 136, H_NTILES = 144, H_NCHUNKS = 152, H_NWORDS = 160,
  H_NEXC = 168, H_NOUT = 176, H_NPATCH = 184, H_BYTES = 192, H_CSUM = 200, H_CONST = 208,
  H_SCALE = 216  // closed loop: factor applied to eb_rel (float64)
};

__host__ __device__ inline uint64_t align8(uint64_t v) { return (v + 7) & ~uint64_t(7); }
__host__ __device__ inline uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// Per-call geometry, computed on the host and passed by value.
struct Plan {
  int32_t ndim, dtype, domain;
  int32_t pad_;                 // 1: some tile is clipped by the field's edge
  uint64_t dims[3];             // as given (slowest-first), unused = 1
  uint64_t nz, ny, nx, n;       // normalized to 3D
  uint32_t tz, ty, tx, pad2_;   // tile extents
  uint32_t gz, gy, gx, pad3_;   // tile grid
  uint64_t n_tiles, n_chunks;
  // blob sections with sizes known before compression
  uint64_t off_len, off_two, off_teo, off_cb, off_exc;
  uint64_t capacity;            // blob capacity (compress) or blob bytes (decompress)
  double target_psnr, eb_rel;
  // closed loop: 10^(-PSNR/10) (host libm), so that the target MSE is
  // vr^2 * mse_factor; closed = 0 for plain compression
  double mse_factor;
  int32_t closed;
  int32_t variant;  // kVarPlain, kVarInloop or kVarXform
};

// Geometry of one tile.
struct TileGeo {
  uint32_t a, b, c;       // tile grid coordinates (z, y, x)
  uint32_t ez, ey, ex;    // clipped extents
  uint64_t z0, y0, x0;    // origin in the field
  uint32_t nt;            // points in the tile
  uint32_t nck;           // chunks in the tile
  uint64_t start;         // stream position of the first point
  uint64_t chunk_base;    // index of the first chunk
};

__host__ __device__ inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

__host__ __device__ inline uint64_t chunks_of(uint64_t ez, uint64_t ey, uint64_t ex) {
  return ceil_div(ez * ey * ex, kChunk);
}

// Closed forms: only the last tile along each axis is clipped, so every tile
// before (a, b, c) in row-major order has full extents along the axes where
// it precedes.
__host__ __device__ inline TileGeo tile_geo(const Plan &P, uint64_t t) {
  TileGeo g;
  // tile counts are below 2^31 (fields hold fewer points): 32-bit divisions,
  // a fraction of the 64-bit sequence on the scalar unit
  const uint32_t t32 = (uint32_t)t, q = t32 / P.gx;
  g.c = t32 - q * P.gx;
  g.a = q / P.gy;
  g.b = q - g.a * P.gy;
  g.z0 = (uint64_t)g.a * P.tz;
  g.y0 = (uint64_t)g.b * P.ty;
  g.x0 = (uint64_t)g.c * P.tx;
  g.ez = (uint32_t)(g.z0 + P.tz <= P.nz ? P.tz : P.nz - g.z0);
  g.ey = (uint32_t)(g.y0 + P.ty <= P.ny ? P.ty : P.ny - g.y0);
  g.ex = (uint32_t)(g.x0 + P.tx <= P.nx ? P.tx : P.nx - g.x0);
  g.nt = g.ez * g.ey * g.ex;
  g.nck = (uint32_t)ceil_div(g.nt, kChunk);
  g.start = g.z0 * P.ny * P.nx + (uint64_t)g.b * g.ez * P.ty * P.nx +
            (uint64_t)g.c * g.ez * g.ey * P.tx;
  const uint64_t ex_last = P.nx - (uint64_t)(P.gx - 1) * P.tx;
  const uint64_t ey_last = P.ny - (uint64_t)(P.gy - 1) * P.ty;
  auto row = [&](uint64_t ez, uint64_t ey) {
    return (uint64_t)(P.gx - 1) * chunks_of(ez, ey, P.tx) + chunks_of(ez, ey, ex_last);
  };
  auto slab = [&](uint64_t ez) { return (uint64_t)(P.gy - 1) * row(ez, P.ty) + row(ez, ey_last); };
  g.chunk_base = (uint64_t)g.a * slab(P.tz) + (uint64_t)g.b * row(g.ez, P.ty) +
                 (uint64_t)g.c * chunks_of(g.ez, g.ey, P.tx);
  return g;
}

// Device parameter / status block, first bytes of every workspace.
struct DevParams {
  uint32_t status;      // fpsz_status of the device-side pipeline
  uint32_t is_const;
  uint32_t big_tiles;   // some tile has more exception records than its staging slot
  uint32_t spin_fail;   // a bounded wait gave up (reported as FPSZ_E_DEVICE)
  uint32_t overflow;    // a blob write fell beyond the capacity
  uint32_t corrupt;     // decompress: inconsistency found
  uint32_t unused_[2];
  double mn, mx, vr, eb_rel, eb, e2, r, maxabs;
  float e2_f, r_f;
  uint64_t nonfinite;
  uint64_t n_out, n_pat, n_exc, off_words, n_words, blob_bytes;
  uint64_t checksum;
  uint64_t verify_done;
  double v_sse, v_max;
  uint64_t v_over;
  double scale;      // closed loop: factor applied to eb_rel (1 otherwise)
  double q_sse;      // closed loop: SSE of the first pass
  uint64_t pad_[6];
};

// ---- wave primitives (wave64) ----------------------------------------------
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// inclusive scan over the 64 lanes
// Inclusive wave scans by DPP (the whole wave must be active): within each
// row of 16 lanes, shifts by 1, 2, 4, 8 (lanes without a source add 0); then
// row 0's total into row 1 and row 2's into row 3 (row_bcast:15), and the
// total of rows 0-1 into rows 2-3 (row_bcast:31).  Each step is a lane move
// inside the ALU, where a shuffle would be a round trip through the LDS
// crossbar.
template <int CTRL, int ROWS, bool BOUND>
__device__ inline uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, BOUND);
}
template <int CTRL, int ROWS, bool BOUND>
__device__ inline void dpp_add_u64(uint64_t &v) {
  const uint32_t lo = dpp_u32<CTRL, ROWS, BOUND>((uint32_t)v);
  const uint32_t hi = dpp_u32<CTRL, ROWS, BOUND>((uint32_t)(v >> 32));
  v += ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t wave_incl_scan_u32(uint32_t v) {
  v += dpp_u32<0x111, 0xf, true>(v);   // row_shr:1
  v += dpp_u32<0x112, 0xf, true>(v);   // row_shr:2
  v += dpp_u32<0x114, 0xf, true>(v);   // row_shr:4
  v += dpp_u32<0x118, 0xf, true>(v);   // row_shr:8
  v += dpp_u32<0x142, 0xa, false>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_u32<0x143, 0xc, false>(v);  // row_bcast:31 into rows 2, 3
  return v;
}
__device__ inline uint64_t wave_incl_scan_u64(uint64_t v) {
  dpp_add_u64<0x111, 0xf, true>(v);
  dpp_add_u64<0x112, 0xf, true>(v);
  dpp_add_u64<0x114, 0xf, true>(v);
  dpp_add_u64<0x118, 0xf, true>(v);
  dpp_add_u64<0x142, 0xa, false>(v);
  dpp_add_u64<0x143, 0xc, false>(v);
  return v;
}

// Block-wide exclusive scan of one u32 per thread (blockDim.x == 256).
// `scratch` holds >= 4 u32.  Returns the exclusive prefix; *total the sum.
__device__ inline uint32_t block_excl_scan_u32(uint32_t v, uint32_t *scratch, uint32_t *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan_u32(v);
  if (lane == 63) scratch[wv] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; w++) {
    uint32_t s = scratch[w];
    if (w < wv) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

__device__ inline uint64_t mix64(uint32_t w, uint64_t j) {
  uint64_t h = (uint64_t)w * 0x9E3779B97F4A7C15ull + j * 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  return h;
}

// Canonical codes from lengths (shared with the decoder-table kernel):
// codes of each length are consecutive in symbol order, and the first code
// of length l is (first(l-1) + count(l-1)) << 1.  A symbol's rank among the
// symbols of its length comes from per-wave ballots over blocks of 64
// symbols.  `wcnt` holds >= 17 * 20 u32.
__device__ inline void canonical_from_lengths(const uint8_t *lens, uint32_t *code_out, uint32_t *lcount,
                                              uint32_t *lfirst, uint32_t *lbase, uint16_t *sorted,
                                              uint32_t *wcnt) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  constexpr int kChunks = (kNSym + 63) / 64;
  uint32_t myrank[2] = {0, 0};
  int k = 0;
  for (int w = wave; w < kChunks; w += nwaves, k++) {
    const int s = 64 * w + lane;
    const int l = s < kNSym ? lens[s] : 0;
    for (int ll = 1; ll <= kLMax; ll++) {
      const uint64_t m = __ballot(l == ll);
      if (lane == 0) wcnt[w * 20 + ll] = (uint32_t)__popcll(m);
      if (l == ll) myrank[k] = (uint32_t)__popcll(m & ((1ull << lane) - 1));
    }
  }
  __syncthreads();
  // thread l - 1 counts the codes of length l over the chunks (in parallel:
  // one thread walking all lengths would chain kLMax * kChunks LDS reads)
  if (tid < kLMax) {
    uint32_t cnt = 0;
    for (int w = 0; w < kChunks; w++) cnt += wcnt[w * 20 + tid + 1];
    lcount[tid + 1] = cnt;
  }
  __syncthreads();
  if (tid == 0) {
    // lcount[0] stays 0: unused symbols are not counted
    uint32_t c = 0, base = 0;
    lcount[0] = 0;
    lfirst[0] = 0;
    lbase[0] = 0;
    for (int l = 1; l <= kLMax; l++) {
      c = (c + lcount[l - 1]) << 1;
      lfirst[l] = c;
      lbase[l] = base;
      base += lcount[l];
    }
  }
  __syncthreads();
  k = 0;
  for (int w = wave; w < kChunks; w += nwaves, k++) {
    const int s = 64 * w + lane;
    if (s >= kNSym) continue;
    const int l = lens[s];
    if (!l) { if (code_out) code_out[s] = 0; continue; }
    uint32_t rank = myrank[k];
    for (int w2 = 0; w2 < w; w2++) rank += wcnt[w2 * 20 + l];
    if (code_out) code_out[s] = lfirst[l] + rank;
    if (sorted) sorted[lbase[l] + rank] = (uint16_t)s;
  }
  __syncthreads();
}

// Checksum workgroups for a blob: about 32 KiB per workgroup (8 rounds of
// 16-byte loads per thread), at most 1024.  Each workgroup ends with a block
// reduction and one atomic; large blobs get more than one per CU to hide the
// hashing's latency.  (128 KiB per workgroup left a 512 x 512 float32 blob
// to a few workgroups looping over it: compression 110 -> 105 us with 32.)
__host__ __device__ inline uint32_t checksum_grid(uint64_t bytes) {
  const uint64_t cw = bytes / (16ull * kBlock * 8) + 1;
  return (uint32_t)(cw < 1024 ? cw : 1024);
}

// checksum over the blob's 32-bit words; the checksum field reads as zero.
// Accumulates into dp->checksum; use_dp_bytes: the blob size is dp->blob_bytes
// (compress, after the header is written), else bytes_limit (decompress).
// Block bi of nb (blocks of any multiple of 64 threads up to 1024).
__device__ inline void checksum_body(const uint8_t *__restrict__ blob, uint64_t bytes_limit,
                                     DevParams *__restrict__ dp, int use_dp_bytes, uint32_t bi,
                                     uint32_t nb) {
  if (use_dp_bytes && (dp->status != 0 || dp->overflow)) return;
  const uint64_t bytes = use_dp_bytes ? dp->blob_bytes : bytes_limit;
  // a grid sized for the capacity uses only the workgroups this blob needs
  const uint32_t want = (checksum_grid(bytes) * kBlock + blockDim.x - 1) / blockDim.x;
  const uint32_t nblk = nb < want ? nb : want;
  if (bi >= nblk) return;  // uniform over the block, before any barrier
  const uint64_t nw = bytes / 4;  // a multiple of 2 (blobs are 8-byte sized)
  const uint32_t *w = reinterpret_cast<const uint32_t *>(blob);
  const uint4 *w4 = reinterpret_cast<const uint4 *>(blob);
  uint64_t s = 0;
  // 16-byte loads when the blob allows them (it is only required to be 8-aligned)
  const uint64_t n4 = (uintptr_t)blob % 16 == 0 ? nw / 4 : 0;
  const uint64_t gsz = (uint64_t)nblk * blockDim.x;
  auto quad = [&](const uint4 v, uint64_t q) {
    const uint64_t j = 4 * q;
    s += mix64(v.x, j) + mix64(v.y, j + 1);
    s += mix64((j + 2 == 50) ? 0u : v.z, j + 2) + mix64((j + 3 == 51) ? 0u : v.w, j + 3);
  };
  uint64_t q = bi * (uint64_t)blockDim.x + threadIdx.x;
  for (; q + 3 * gsz < n4; q += 4 * gsz) {  // four loads in flight per thread
    const uint4 a = w4[q], b = w4[q + gsz], c = w4[q + 2 * gsz], d = w4[q + 3 * gsz];
    quad(a, q);
    quad(b, q + gsz);
    quad(c, q + 2 * gsz);
    quad(d, q + 3 * gsz);
  }
  for (; q < n4; q += gsz) quad(w4[q], q);
  for (uint64_t j = n4 * 4 + bi * (uint64_t)blockDim.x + threadIdx.x; j < nw; j += gsz)
    s += mix64((j == 50 || j == 51) ? 0u : w[j], j);
  // one atomic per block: atomics on one address are serialized, so their
  // count, not the memory traffic, would set the kernel's time
  __shared__ uint64_t part[16];
  s = wave_sum_u64(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t b = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) b += part[i];
    if (b) atomicAdd((unsigned long long *)&dp->checksum, (unsigned long long)b);
  }
}

// Optional per-stage timing with HIP events recorded on the launch stream.
struct Timer {
  static constexpr int kMax = 48;
  bool on = false;
  int n = 0;
  hipEvent_t ev[kMax];
  const char *names[kMax];
  void mark(hipStream_t s, const char *name) {
    if (on && n < kMax) {
      names[n] = name;
      (void)hipEventRecord(ev[n], s);
      n++;
    }
  }
};

// ---- launchers (defined in the .hip files) ---------------------------------
struct CompressWs {
  DevParams *P;
  void *range_part;
  uint32_t *hist;
  uint8_t *code_len;
  uint32_t *code;
  uint32_t *exc_cnt;    // per-tile exception record counts
  uint64_t *exc_off;    // per-tile record offsets
  uint32_t *stage;      // staged records, kStage per tile
  uint64_t *word_state;
  uint8_t *code_w8;     // per tile and wave: its residual codes stored as int8 (1) or int16 (0)
  int16_t *codes;
  uint64_t zero_bytes;  // bytes from P to clear before a call
};

struct DecompressWs {
  DevParams *P;
  uint16_t *lut;       // 8192 entries: (symbol << 5) | length, 0 = long/invalid
  uint32_t *ltab;      // first[19], count[19], base[19]
  uint16_t *sorted;    // symbols in canonical order
  uint32_t *fz, *fy, *fx;  // per-tile faces (GLOBAL domain)
  uint32_t *gx, *gy, *gz, *tt;  // per-tile edge vectors and totals
  uint32_t *tmp;           // segment sums of the scans
  int16_t *codes;          // decoded residual codes, stream order
  uint8_t *res8;           // one-launch decompression: 32-code parts stored as int8, stream order
  uint64_t *res8_mask;     // per tile, mask p: bit L set when part 4 L + p is in res8
  double *vpart;           // check against the original: per-tile (sse, max |e|, count > eb)
  uint64_t zero_bytes;
};

// One field of a compress launch.  Kernels take a job by value (a single
// field) and a device array of jobs indexed by blockIdx.y (a batched launch
// over many fields); a null array selects the by-value job.  Every field of a
// batched launch has the same dtype, ndim and Lorenzo domain (the kernel's
// template class); sizes and targets may differ.
struct CJob {
  Plan P;
  const void *x;
  CompressWs W;
  uint8_t *blob;
};

// Launch shape of the compress kernels (grid x per field).  None of these
// changes a single output bit: tiles are fixed by the format, every
// reduction is order-independent or has a fixed order.
struct LaunchCfg {
  uint32_t range_blocks;  // k_range blocks per field
  uint32_t quant_grid;    // k_quant workgroups per field (persistent over tiles)
  uint32_t encode_grid;   // k_encode workgroups per field (tickets over tiles)
  uint32_t csum_blocks;   // k_checksum blocks per field
};
LaunchCfg default_launch_cfg(const Plan &maxP);

// Launch the whole compress pipeline for `nf` fields (nf == 1 and jobs_dev ==
// nullptr: the single field `one`).  maxP carries the class (dtype, ndim,
// domain) and the largest n / n_tiles / capacity of the fields.
hipError_t launch_compress_jobs(const CJob &one, const CJob *jobs_dev, int nf, const Plan &maxP,
                                const LaunchCfg &cfg, hipStream_t s, Timer *tm);

hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t s);
// a blob header expected in device memory (the caller's host copy)
struct HdrBytes {
  uint32_t w[64];
};
hipError_t launch_hdr_check(const uint8_t *blob, const HdrBytes &h, DevParams *dp, hipStream_t s);
// fpsz_decompress_async's outcome
hipError_t launch_dasync_result(DevParams *dp, fpsz_decompress_result *out, int is_const,
                                uint64_t csum, int checked, uint64_t n, double vr, hipStream_t s);
// the outcome of a compression into a device-side fpsz_async_result
hipError_t launch_async_result(const CJob &one, fpsz_async_result *out, hipStream_t s);
hipError_t launch_decompress_args(const Plan &P, const uint8_t *blob, const DecompressWs &W,
                                  uint64_t off_words, uint64_t n_words, uint64_t n_exc, double e2,
                                  float e2_f, void *out, const void *ref, double eb, hipStream_t s,
                                  Timer *tm, const HdrBytes *hdr = nullptr);
hipError_t launch_const_fill_bits(const Plan &P, uint64_t bits, void *out, hipStream_t s);
hipError_t launch_checksum(const uint8_t *blob, uint64_t bytes, DevParams *dp, hipStream_t s);
hipError_t launch_verify(const void *x, const void *y, uint64_t n, int dtype, double eb,
                         DevParams *P, void *part, hipStream_t s, Timer *tm);

}  // namespace fpsz
