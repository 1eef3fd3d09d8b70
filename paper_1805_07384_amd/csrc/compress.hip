// compress.hip -- gfx950 kernels of fixed-PSNR SZ-style compression.
//
// Pipeline (one stream, no host round trip until the end):
//   k_range, k_range_final  value range of the original data (definition
//               under Eq. 4) from per-block partials, then eb_abs =
//               eb_rel * vr (Eq. 7, remark after Eq. 6), the bin size 2 eb
//               and its reciprocal; the range blocks also clear the call's
//               parameter block and counters
//   k_quant     prequantization q = rint(x / 2eb) (uniform bins with
//               midpoint reconstruction, Eq. 5-6), Lorenzo residual on q
//               from an LDS tile with a one-point halo (Sec. II-A step (1),
//               Sec. III), symbol histogram, residual codes, and the tile's
//               exception records staged in stream order
//   k_codebook  Huffman code lengths (Sec. II-A step (2)) and canonical
//               codes; a second workgroup scans the tiles' record counts
//   k_enc_count, k_enc_scan, k_enc_pack  bits per chunk and tile, the
//               tiles' word offsets (and the header), the bit packing
//   k_checksum_jobs, k_checksum_store  the blob checksum
#include <float.h>
#include <math.h>

#include "fpsz_internal.h"

namespace fpsz {

// ---------------------------------------------------------------------------
// The field a block works on: the by-value job, or entry blockIdx.y of the
// batch array.
// The copy is made wave-uniform word by word, so everything derived from it
// (tile geometry, addresses) stays in scalar registers.
__device__ inline CJob select_job(const CJob &one, const CJob *__restrict__ jobs) {
  CJob j;
  if (jobs) j = jobs[blockIdx.y];
  else j = one;
  static_assert(sizeof(CJob) % 4 == 0, "CJob is copied in 32-bit words");
  uint32_t w[sizeof(CJob) / 4];
  __builtin_memcpy(w, &j, sizeof(CJob));
#pragma unroll
  for (unsigned i = 0; i < sizeof(CJob) / 4; i++) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  __builtin_memcpy(&j, w, sizeof(CJob));
  return j;
}

__global__ void k_fill_zero(uint32_t *p, uint64_t nwords) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nwords;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t s) {
  const uint64_t nw = bytes / 4;
  if (nw == 0) return hipSuccess;
  const uint64_t blocks = nw / kBlock + 1 < 1024 ? nw / kBlock + 1 : 1024;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint32_t *)p, nw);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a1: range reduction.  Each block reduces a grid-stride share into a
// partial; one block per field combines the partials and derives the error
// bound.  (No block waits on another and no atomics: a counter on one
// address serializes every block that reaches it.)  The range blocks also
// clear the field's parameter block, histograms, code tables and tile word
// counts for the rest of the call (the first launch of a compression; no
// kernel of it reads them, and the partials they write are not cleared).
typedef float rf32x4_t __attribute__((ext_vector_type(4)));
typedef double rf64x2_t __attribute__((ext_vector_type(2)));
template <typename T> struct VecOf;
template <> struct VecOf<float> { using V = rf32x4_t; static constexpr int W = 4; };
template <> struct VecOf<double> { using V = rf64x2_t; static constexpr int W = 2; };

__device__ inline bool finite_f(float v) { return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u; }
__device__ inline bool finite_f(double v) {
  return ((unsigned long long)__double_as_longlong(v) & 0x7ff0000000000000ull) != 0x7ff0000000000000ull;
}

// Branch-free: a non-finite value is counted (the field is then rejected,
// so what min / max make of it does not matter).
__device__ inline void acc_range(float v, float &mn, float &mx, uint32_t &bad) {
  bad += finite_f(v) ? 0u : 1u;
  mn = __builtin_fminf(mn, v);
  mx = __builtin_fmaxf(mx, v);
}
__device__ inline void acc_range(double v, double &mn, double &mx, uint32_t &bad) {
  bad += finite_f(v) ? 0u : 1u;
  mn = __builtin_fmin(mn, v);
  mx = __builtin_fmax(mx, v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_range(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const T *__restrict__ x = static_cast<const T *>(J.x);
  const Plan P = J.P;
  uint64_t *__restrict__ part = static_cast<uint64_t *>(J.W.range_part);
  using V = typename VecOf<T>::V;
  typedef __attribute__((address_space(1))) const V gV;
  typedef __attribute__((address_space(1))) const T gT;
  constexpr int W = VecOf<T>::W;
  const uint64_t n = P.n;
  T mn = (T)INFINITY, mx = (T)-INFINITY;
  uint32_t bad = 0;
  // unaligned head (at most W - 1 elements) and tail handled element-wise
  const uint64_t mis = ((uintptr_t)x / sizeof(T)) % W;
  const uint64_t head = mis ? (W - mis < n ? W - mis : n) : 0;
  const uint64_t nvec = (n - head) / W;
  const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t gsz = (uint64_t)gridDim.x * blockDim.x;
  {
    uint32_t *z = reinterpret_cast<uint32_t *>(J.W.P);
    const uint64_t a = (uint64_t)(reinterpret_cast<const uint8_t *>(J.W.range_part) -
                                  reinterpret_cast<const uint8_t *>(J.W.P)) / 4;
    const uint64_t b = (uint64_t)(reinterpret_cast<const uint8_t *>(J.W.hist) -
                                  reinterpret_cast<const uint8_t *>(J.W.P)) / 4;
    const uint64_t nw = J.W.zero_bytes / 4;
    for (uint64_t i = gtid; i < a; i += gsz) z[i] = 0;
    for (uint64_t i = b + gtid; i < nw; i += gsz) z[i] = 0;
  }
  gV *xv = (gV *)(x + head);
  uint64_t i = gtid;
  for (; i + 7 * gsz < nvec; i += 8 * gsz) {  // eight 16-byte loads in flight
    V a[8];
#pragma unroll
    for (int u = 0; u < 8; u++) a[u] = xv[i + u * gsz];
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int k = 0; k < W; k++) acc_range((T)a[u][k], mn, mx, bad);
  }
  for (; i < nvec; i += gsz) {
    const V a = xv[i];
#pragma unroll
    for (int k = 0; k < W; k++) acc_range((T)a[k], mn, mx, bad);
  }
  if (gtid < head) acc_range(((gT *)x)[gtid], mn, mx, bad);
  const uint64_t tail0 = head + nvec * W;
  if (gtid < n - tail0) acc_range(((gT *)x)[tail0 + gtid], mn, mx, bad);

  // block partial
  double dmn = (double)mn, dmx = (double)mx;
  uint64_t dbad = bad;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double a = __shfl_xor(dmn, o, 64), b = __shfl_xor(dmx, o, 64);
    dmn = __builtin_fmin(dmn, a);
    dmx = __builtin_fmax(dmx, b);
    dbad += __shfl_xor(dbad, o, 64);
  }
  __shared__ double smn[kBlock / 64], smx[kBlock / 64];
  __shared__ uint64_t sbad[kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { smn[wv] = dmn; smx[wv] = dmx; sbad[wv] = dbad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; w++) {
      dmn = __builtin_fmin(dmn, smn[w]);
      dmx = __builtin_fmax(dmx, smx[w]);
      dbad += sbad[w];
    }
    part[3 * blockIdx.x + 0] = (uint64_t)__double_as_longlong(dmn);
    part[3 * blockIdx.x + 1] = (uint64_t)__double_as_longlong(dmx);
    part[3 * blockIdx.x + 2] = dbad;
  }
}

// eb_abs = eb_rel * vr (Eq. 7 and the remark after Eq. 6), the bin size 2 eb,
// its reciprocal and the range guard
__device__ inline void derive_bound(const Plan &P, DevParams *dp, double vr, double eb_rel) {
  const double eb = vr * eb_rel;
  const double e2 = 2.0 * eb;
  const double r = 1.0 / e2;
  dp->vr = vr;
  dp->eb_rel = eb_rel;
  dp->eb = eb;
  dp->e2 = e2;
  dp->r = r;
  dp->e2_f = (float)e2;
  dp->r_f = (float)r;
  const double maxabs = fabs(dp->mn) > fabs(dp->mx) ? fabs(dp->mn) : fabs(dp->mx);
  dp->maxabs = maxabs;
  if (vr == 0.0) { dp->is_const = 1; return; }
  const double lim = P.dtype == FPSZ_F32 ? 8388608.0 : 134217728.0;
  if (!(maxabs * r < lim)) dp->status = FPSZ_E_RANGE;
}

// one block per field: combine the nb partials, derive eb (Eq. 7) and the
// quantizer constants
__global__ __launch_bounds__(kBlock) void k_range_final(CJob one, const CJob *__restrict__ jobs,
                                                        uint32_t nb) {
  const CJob J = select_job(one, jobs);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  const uint64_t *__restrict__ part = static_cast<const uint64_t *>(J.W.range_part);
  double bmn = INFINITY, bmx = -INFINITY;
  uint64_t bbad = 0;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    bmn = __builtin_fmin(bmn, __longlong_as_double((long long)part[3 * b + 0]));
    bmx = __builtin_fmax(bmx, __longlong_as_double((long long)part[3 * b + 1]));
    bbad += part[3 * b + 2];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double a = __shfl_xor(bmn, o, 64), c = __shfl_xor(bmx, o, 64);
    bmn = __builtin_fmin(bmn, a);
    bmx = __builtin_fmax(bmx, c);
    bbad += __shfl_xor(bbad, o, 64);
  }
  __shared__ double smn[kBlock / 64], smx[kBlock / 64];
  __shared__ uint64_t sbad[kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { smn[wv] = bmn; smx[wv] = bmx; sbad[wv] = bbad; }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < kBlock / 64; w++) {
    bmn = __builtin_fmin(bmn, smn[w]);
    bmx = __builtin_fmax(bmx, smx[w]);
    bbad += sbad[w];
  }
  dp->nonfinite = bbad;
  if (bbad) { dp->status = FPSZ_E_NONFINITE; return; }
  const double vmn = bmn + 0.0, vmx = bmx + 0.0;  // -0 reads as +0
  dp->mn = vmn;
  dp->mx = vmx;
  dp->scale = 1.0;
  derive_bound(P, dp, vmx - vmn, P.eb_rel);
}


// ---------------------------------------------------------------------------
// a3-a7: prequantization, Lorenzo residual, symbols, histogram, codes and
// the exception list.
//
// The tile and its one-point halo (the preceding plane, row and column) are
// quantized into an LDS box.  Rows of the box are loaded by one thread each
// (segments of up to 32 points along x), so the index arithmetic is paid per
// row, not per point.  Each thread then owns 32 consecutive points of the
// stream and walks them along x, reusing the previous point's neighbours.
// Exception records of a tile (outliers, then patches, in stream order) are
// staged in a fixed slot of kStage records; a later pass places them at
// their final offsets (tiles with more records recompute them there).
template <int NDIM> struct Geo;
template <> struct Geo<1> { static constexpr int TZ = 1, TY = 1, TX = 8192, HZ = 0, HY = 0; };
template <> struct Geo<2> { static constexpr int TZ = 1, TY = 64, TX = 128, HZ = 0, HY = 1; };
template <> struct Geo<3> { static constexpr int TZ = 16, TY = 16, TX = 32, HZ = 1, HY = 1; };

// LDS address of box point (bz, by, bx): rows of TX + 1 points; the 1D box
// (a single long row) gets one pad word per 32 points to spread banks.
template <int NDIM> struct BoxAddr {
  using G = Geo<NDIM>;
  static constexpr int BZ = G::TZ + G::HZ, BY = G::TY + G::HY, BX = G::TX + 1;
  static constexpr int BOX = BZ * BY * BX;
  static constexpr int SIZE = NDIM == 1 ? BOX + (BOX >> 5) + 1 : BOX;
  __device__ static int at(int bz, int by, int bx) {
    const int L = (bz * BY + by) * BX + bx;
    return NDIM == 1 ? L + (L >> 5) : L;
  }
};

template <typename T> struct Quant;
template <> struct Quant<float> {
  __device__ static int32_t q(float v, float rf, double) { return (int32_t)__builtin_rintf(v * rf); }
  __device__ static bool patch(float v, int32_t q, float e2f, double, double eb) {
    const float xr = (float)q * e2f;
    return fabs((double)v - (double)xr) > eb;
  }
};
template <> struct Quant<double> {
  __device__ static int32_t q(double v, float, double r) { return (int32_t)__builtin_rint(v * r); }
  __device__ static bool patch(double v, int32_t q, float, double e2, double eb) {
    const double xr = (double)q * e2;
    return fabs(v - xr) > eb;
  }
};

constexpr int kStage = 64;  // staged exception records per tile

// Load one box row segment: points bx in [1 + 32 seg, 1 + 32 seg + 32) of box
// row (bz, by), plus the halo point bx = 0 when seg == 0.  Quantizes into
// the box and sets patch bits of interior points.
template <typename T, int NDIM, bool GLOBAL>
__device__ inline void load_row(const T *__restrict__ x, const Plan &P, const TileGeo &g, int bz,
                                int by, int seg, int32_t *box, uint32_t *pmask, float rf, double r,
                                float e2f, double e2, double eb) {
  using G = Geo<NDIM>;
  using B = BoxAddr<NDIM>;
  const int z = bz - G::HZ, y = by - G::HY;
  const int ez = (int)g.ez, ey = (int)g.ey, ex = (int)g.ex;
  const bool row_in = z < ez && y < ey;
  const bool row_field = GLOBAL ? ((z >= 0 || g.z0 > 0) && (y >= 0 || g.y0 > 0)) : (z >= 0 && y >= 0);
  const bool interior_row = z >= 0 && y >= 0;
  const int x0l = 32 * seg;  // first interior x (tile-local) of the segment
  int nx_seg = ex - x0l;
  nx_seg = nx_seg < 0 ? 0 : (nx_seg > 32 ? 32 : nx_seg);
  const bool load_row_pts = row_in && row_field;
  const uint64_t rowbase =
      ((uint64_t)((int64_t)g.z0 + z) * P.ny + (uint64_t)((int64_t)g.y0 + y)) * P.nx + g.x0;
  // halo column point (x0 - 1)
  if (seg == 0) {
    int32_t qh = 0;
    if (GLOBAL && load_row_pts && g.x0 > 0) qh = Quant<T>::q(x[rowbase - 1], rf, r);
    box[B::at(bz, by, 0)] = qh;
  }
  T v[32];
  constexpr int VW = 16 / sizeof(T);
  const bool vec = load_row_pts && nx_seg == 32 && (((rowbase + x0l) % VW) == 0);
  if (vec) {
    using V = typename VecOf<T>::V;
    const V *src = reinterpret_cast<const V *>(x + rowbase + x0l);
#pragma unroll
    for (int k = 0; k < 32 / VW; k++) {
      const V a = src[k];
      const T *pa = reinterpret_cast<const T *>(&a);
#pragma unroll
      for (int h = 0; h < VW; h++) v[k * VW + h] = pa[h];
    }
  } else if (load_row_pts && nx_seg > 0) {
    // Inside the field buffer the segment is read whole (points past the
    // tile's edge are the next row's, masked below): 32 loads from one
    // address, issued before any is waited for.  Written as
    // j < nx_seg ? x[..] : 0 each load got its own branch and wait, which is
    // left to the segments that end the buffer.
    const T *src = x + rowbase + x0l;
    if (rowbase + x0l + 32 <= P.n) {
#pragma unroll
      for (int j = 0; j < 32; j++) v[j] = src[j];
#pragma unroll
      for (int j = 0; j < 32; j++) v[j] = j < nx_seg ? v[j] : (T)0;
    } else {
#pragma unroll
      for (int j = 0; j < 32; j++) v[j] = j < nx_seg ? src[j] : (T)0;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 32; j++) v[j] = (T)0;
  }
  uint32_t pbits = 0;
#pragma unroll
  for (int j = 0; j < 32; j++) {
    const int32_t qv = Quant<T>::q(v[j], rf, r);
    if (row_in && j < nx_seg) box[B::at(bz, by, 1 + x0l + j)] = qv;
    if (interior_row && row_in && j < nx_seg && Quant<T>::patch(v[j], qv, e2f, e2, eb))
      pbits |= 1u << j;
  }
  if (pbits) {
    // stream index of the segment's first point
    const int si = (z * ey + y) * ex + x0l;
    const int w = si >> 5, sh = si & 31;
    atomicOr(&pmask[w], pbits << sh);
    if (sh) atomicOr(&pmask[w + 1], pbits >> (32 - sh));
  }
}

// Full tiles (the common case) take a leaner path: each thread owns one
// 32-point row segment of the stream, loads it with 16-byte loads, keeps its
// q in registers and computes its patch bits directly.  LDS holds the q
// segments of the tile and of the halo (the preceding plane and row), each
// padded to kSegW words with its left neighbour just before the 16-byte
// aligned values, so a neighbouring segment is 8 + 1 LDS reads without bank
// conflicts.  The halo points are loaded by all threads together.
constexpr int kSegW = 36;
template <int NDIM> struct FastGeo;
template <> struct FastGeo<1> { static constexpr int NSEG = 256, HROWS = 0, ROWS = 1; };
template <> struct FastGeo<2> { static constexpr int NSEG = 4, HROWS = 1, ROWS = 65; };
template <> struct FastGeo<3> { static constexpr int NSEG = 1, HROWS = 33, ROWS = 17 * 17; };

// LDS word of value k (k = -1 is the left neighbour) of segment s of box row
// (bz, by) (box coordinates include the halo)
template <int NDIM> __device__ inline int seg_at(int bz, int by, int s, int k) {
  using G = Geo<NDIM>;
  const int row = bz * (G::TY + G::HY) + by;
  return (row * FastGeo<NDIM>::NSEG + s) * kSegW + 4 + k;
}

// Patch test |x - x'| > eb.  For float32 input a float32 pre-filter marks
// candidates: below thr (eb lowered by a relative 2^-22, rounded down) the
// rounded float32 difference proves |x - x'| <= eb; candidates (rare) take
// the exact float64 test afterwards.  Full tiles keep only the largest
// difference of a 32-point segment and test every point of a segment above
// thr exactly.
template <typename T> struct PatchTest;
template <> struct PatchTest<float> {
  // |x - x'| rounded to float32 (x' itself rounded first, as the decoder
  // forms it)
  __device__ static float diff(float v, int32_t q, float e2f) {
    const float xr = (float)q * e2f;
    return fabsf(v - xr);
  }
  __device__ static bool candidate(float v, int32_t q, float e2f, double, double, float thr) {
    return diff(v, q, e2f) > thr;
  }
  __device__ static bool exact(float v, int32_t q, float e2f, double, double eb) {
    const float xr = (float)q * e2f;
    return fabs((double)v - (double)xr) > eb;
  }
};
template <> struct PatchTest<double> {
  __device__ static bool candidate(double v, int32_t q, float, double e2, double eb, float) {
    return fabs(v - (double)q * e2) > eb;
  }
  __device__ static bool exact(double v, int32_t q, float, double e2, double eb) {
    return fabs(v - (double)q * e2) > eb;
  }
};

// global-memory views of the input (the pointers reach the kernels inside
// job structures, where the compiler cannot see their address space)
template <typename T> using gptr_t = __attribute__((address_space(1))) const T *;
typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
template <typename T> struct GVec;
template <> struct GVec<float> { using V = f32x4_t; };
template <> struct GVec<double> { using V = f64x2_t; };

// Closed loop, first pass: SSE of the quantizer's output at the Eq. 7 bound
// (by Theorem 1 the reconstruction error; a patch is stored exactly and adds
// nothing).  Block b reduces a fixed grid-stride share in a fixed order into
// part[b] (the range partials are free once k_range_final has run).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_qerr(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const Plan P = J.P;
  const DevParams *__restrict__ dp = J.W.P;
  double *__restrict__ part = static_cast<double *>(J.W.range_part);
  if (!P.closed || dp->status != 0 || dp->is_const) return;
  const T *__restrict__ x = static_cast<const T *>(J.x);
  const float rf = dp->r_f, e2f = dp->e2_f;
  const double r = dp->r, e2 = dp->e2, eb = dp->eb;
  double sse = 0.0;
  const uint64_t gsz = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < P.n; i += gsz) {
    const T v = ((gptr_t<T>)x)[i];
    const int32_t q = Quant<T>::q(v, rf, r);
    double e;
    if constexpr (sizeof(T) == 4) e = (double)v - (double)((float)q * e2f);
    else e = v - (double)q * e2;
    e = fabs(e) > eb ? 0.0 : e;
    sse = __builtin_fma(e, e, sse);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sse += __shfl_xor(sse, o, 64);
  __shared__ double s_w[kBlock / 64];
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = sse;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

// Closed loop, the step (one block per field): MSE_1 from the partials in a
// fixed order, the target MSE that Eq. 4 maps to the target PSNR,
// MSE_t = vr^2 10^(-PSNR/10), and the secant factor sqrt(MSE_t / MSE_1) on
// MSE ~ eb^2 (Eq. 6); the bound and quantizer constants are derived again
// from eb_rel times that factor.
__global__ __launch_bounds__(kBlock) void k_rescale(CJob one, const CJob *__restrict__ jobs,
                                                    uint32_t nb) {
  const CJob J = select_job(one, jobs);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  const double *__restrict__ part = static_cast<const double *>(J.W.range_part);
  if (!P.closed || dp->status != 0 || dp->is_const) return;
  double sse = 0.0;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) sse += part[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sse += __shfl_xor(sse, o, 64);
  __shared__ double s_w[kBlock / 64];
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = sse;
  __syncthreads();
  if (threadIdx.x != 0) return;
  sse = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
  dp->q_sse = sse;
  if (!(sse > 0.0)) return;  // the first pass is exact: factor 1
  const double vr = dp->vr;
  const double mse_t = vr * vr * P.mse_factor;
  const double scale = sqrt(mse_t / (sse / (double)P.n));
  dp->scale = scale;
  derive_bound(P, dp, vr, P.eb_rel * scale);
}

// Full tile, phase 1: quantize this thread's segment (and its left
// neighbour) into LDS, the halo points with the other threads; patch bits of
// the segment.  Ends with the LDS written, before the barrier.
template <typename T, int NDIM, bool GLOBAL>
__device__ inline uint32_t fast_tile_load(const T *__restrict__ x_, const Plan &P,
                                          const TileGeo &g, int tid, int32_t *lds, float rf,
                                          double r, float e2f, double e2, double eb, float thr) {
  using G = Geo<NDIM>;
  using F = FastGeo<NDIM>;
  gptr_t<T> x = (gptr_t<T>)x_;
  const int z = NDIM == 3 ? tid >> 4 : 0;
  const int y = NDIM == 3 ? tid & 15 : NDIM == 2 ? tid >> 2 : 0;
  const int sg = NDIM == 3 ? 0 : NDIM == 2 ? tid & 3 : tid;
  const int x0l = 32 * sg;
  const uint32_t rowbase = (((uint32_t)g.z0 + z) * (uint32_t)P.ny + ((uint32_t)g.y0 + y)) *
                               (uint32_t)P.nx + (uint32_t)g.x0 + x0l;
  T v[32];
  constexpr int VW = 16 / sizeof(T);
  if ((rowbase % VW) == 0) {
    using V = typename GVec<T>::V;
    gptr_t<V> src = (gptr_t<V>)(x + rowbase);
#pragma unroll
    for (int k = 0; k < 32 / VW; k++) {
      const V a = src[k];
#pragma unroll
      for (int h = 0; h < VW; h++) v[k * VW + h] = a[h];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 32; j++) v[j] = x[rowbase + j];
  }
  // left neighbour of the segment
  const bool hasl = x0l > 0 || (GLOBAL && g.x0 > 0);
  const T xl = hasl ? x[rowbase - 1] : (T)0;
  // halo rows: 3D the plane z = -1 (17 rows) and the rows y = -1 of z >= 0
  // (16 rows); 2D the row y = -1; 33 values per segment (k = -1 .. 31).
  // All of a thread's halo values are loaded before any is used, so their
  // latencies overlap.
  constexpr int NH = F::HROWS * F::NSEG * 33;
  constexpr int NIT = (NH + kBlock - 1) / kBlock;
  T hv[NIT > 0 ? NIT : 1];
  int hs[NIT > 0 ? NIT : 1];  // LDS word, -1: none
  bool hin[NIT > 0 ? NIT : 1];
#pragma unroll
  for (int m = 0; m < NIT; m++) {
    const int i = tid + m * kBlock;
    const int hr = i / (F::NSEG * 33), rem = i - hr * (F::NSEG * 33);
    const int s2 = rem / 33, k = rem - s2 * 33 - 1;
    const int bz = NDIM == 3 ? (hr < 17 ? 0 : hr - 16) : 0;
    const int by = NDIM == 3 ? (hr < 17 ? hr : 0) : 0;
    hs[m] = i < NH ? seg_at<NDIM>(bz, by, s2, k) : -1;
    hin[m] = false;
    hv[m] = (T)0;
    if (GLOBAL && i < NH) {
      // fields hold fewer than 2^31 points: 32-bit element indexes
      const int32_t fz = (int32_t)g.z0 + bz - G::HZ, fy = (int32_t)g.y0 + by - G::HY;
      const int32_t fx = (int32_t)g.x0 + 32 * s2 + k;
      hin[m] = fz >= 0 && fy >= 0 && fx >= 0;
      const uint32_t fi = ((uint32_t)fz * (uint32_t)P.ny + (uint32_t)fy) * (uint32_t)P.nx + (uint32_t)fx;
      if (hin[m]) hv[m] = x[fi];
    }
  }
  int32_t *dst = lds + seg_at<NDIM>(z + G::HZ, y + G::HY, sg, 0);
  dst[-1] = hasl ? Quant<T>::q(xl, rf, r) : 0;
  uint32_t cand = 0;
  float dmax = 0.0f;  // float input: the largest pre-filter difference
#pragma unroll
  for (int k = 0; k < 8; k++) {
    int32_t q4[4];
#pragma unroll
    for (int h = 0; h < 4; h++) {
      const int j = 4 * k + h;
      q4[h] = Quant<T>::q(v[j], rf, r);
      if constexpr (sizeof(T) == 4)
        dmax = fmaxf(dmax, PatchTest<T>::diff(v[j], q4[h], e2f));
      else
        cand |= (PatchTest<T>::candidate(v[j], q4[h], e2f, e2, eb, thr) ? 1u : 0u) << j;
    }
    reinterpret_cast<int4 *>(dst)[k] = make_int4(q4[0], q4[1], q4[2], q4[3]);
  }
  uint32_t pb = 0;
  if constexpr (sizeof(T) == 4) {
    if (dmax > thr) {
      // rare: every point of the segment takes the exact test, the values
      // reloaded together and quantized again (so no quantized value has
      // to stay in a register for this)
      T w[32];
      if ((rowbase % VW) == 0) {
        using V = typename GVec<T>::V;
        gptr_t<V> src = (gptr_t<V>)(x + rowbase);
#pragma unroll
        for (int k = 0; k < 32 / VW; k++) {
          const V a = src[k];
#pragma unroll
          for (int h = 0; h < VW; h++) w[k * VW + h] = a[h];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 32; j++) w[j] = x[rowbase + j];
      }
#pragma unroll
      for (int j = 0; j < 32; j++)
        pb |= (PatchTest<T>::exact(w[j], Quant<T>::q(w[j], rf, r), e2f, e2, eb) ? 1u : 0u) << j;
    }
  } else {
    // rare: exact test of each candidate, the value reloaded
#pragma unroll 1
    while (cand) {
      const int j = __ffs(cand) - 1;
      cand &= cand - 1;
      const T xv = x[rowbase + j];
      if (PatchTest<T>::exact(xv, Quant<T>::q(xv, rf, r), e2f, e2, eb)) pb |= 1u << j;
    }
  }
#pragma unroll
  for (int m = 0; m < NIT; m++)
    if (hs[m] >= 0) lds[hs[m]] = hin[m] ? Quant<T>::q(hv[m], rf, r) : 0;
  return pb;
}

// LDS pointers of this thread's segment and its y, z, (z, y) neighbours
template <int NDIM> struct SegPtrs {
  const int32_t *o, *y, *z, *zy;
  __device__ SegPtrs(const int32_t *lds, int tid) {
    using G = Geo<NDIM>;
    const int z_ = NDIM == 3 ? tid >> 4 : 0;
    const int y_ = NDIM == 3 ? tid & 15 : NDIM == 2 ? tid >> 2 : 0;
    const int sg = NDIM == 3 ? 0 : NDIM == 2 ? tid & 3 : tid;
    o = lds + seg_at<NDIM>(z_ + G::HZ, y_ + G::HY, sg, 0);
    y = NDIM >= 2 ? lds + seg_at<NDIM>(z_ + G::HZ, y_ + G::HY - 1, sg, 0) : o;
    z = NDIM == 3 ? lds + seg_at<NDIM>(z_ + G::HZ - 1, y_ + G::HY, sg, 0) : o;
    zy = NDIM == 3 ? lds + seg_at<NDIM>(z_ + G::HZ - 1, y_ + G::HY - 1, sg, 0) : o;
  }
  // residual of point j (0..31) of the segment
  __device__ int32_t d_at(int j) const {
    int32_t dv = o[j] - o[j - 1];
    if (NDIM >= 2) dv -= y[j] - y[j - 1];
    if (NDIM == 3) dv += (zy[j] - zy[j - 1]) - (z[j] - z[j - 1]);
    return dv;
  }
};

// Symbol of residual d (|d| <= 511 direct, escape classes, 0 = outlier)
__device__ inline uint32_t symbol_of(int32_t dv, bool &outlier) {
  const int32_t a = dv < 0 ? -dv : dv;
  outlier = a >= 32768;
  const uint32_t esc = 1024u + 2u * (uint32_t)(22 - __clz(a)) + (dv < 0 ? 1u : 0u);
  return a <= 511 ? (uint32_t)(dv + 512) : (outlier ? 0u : esc);
}

// Tile order of the persistent quantization grids.  Workgroups are
// dispatched round-robin over the 8 XCDs (each with its own L2), so block b
// runs on XCD b % 8.  With halos to read (GLOBAL domain) and a tile-row count
// along y that splits evenly over the XCDs (16 or more rows, a multiple of
// 8), XCD x owns the band of tile rows b in [x gy / 8, (x + 1) gy / 8) and
// walks it z-major, then row, then x: the tile before along z (one
// band-layer earlier), along y (one row earlier) and along x (just before)
// were all loaded by the same XCD shortly before, so the halo the tile
// reads is still in that XCD's L2.  Otherwise tiles go round-robin over the
// workgroups (bands of unequal size would leave XCDs idle: 29 tile rows give
// bands of 3 and 4).
__device__ inline bool xcd_tile(const Plan &P, int ndim, uint64_t k, uint64_t *t, bool halo) {
  if (!halo || (gridDim.x & 7) != 0 || ndim < 2 || P.gy < 16 || (P.gy & 7) != 0) {
    *t = blockIdx.x + k * gridDim.x;
    return *t < P.n_tiles;
  }
  // tile counts are below 2^31: 32-bit divisions
  const uint32_t x = blockIdx.x & 7;
  const uint32_t b0 = x * P.gy / 8, b1 = (x + 1) * P.gy / 8;
  const uint32_t row = (b1 - b0) * P.gx;  // tiles of one band-layer
  const uint64_t L64 = (blockIdx.x >> 3) + k * (gridDim.x >> 3);
  if (L64 >= (uint64_t)row * P.gz) return false;
  const uint32_t L = (uint32_t)L64, a = L / row, rem = L - a * row;
  const uint32_t rr = rem / P.gx;
  *t = ((uint64_t)a * P.gy + b0 + rr) * P.gx + (rem - rr * P.gx);
  return true;
}

template <typename T, int NDIM, bool GLOBAL, bool RECORDS, bool FULL>
__global__ __launch_bounds__(kBlock) void k_quant(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const T *__restrict__ x = static_cast<const T *>(J.x);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  uint32_t *__restrict__ hist_g = J.W.hist;
  uint32_t *__restrict__ exc_cnt = J.W.exc_cnt;
  uint32_t *__restrict__ stage = J.W.stage;
  const uint64_t *__restrict__ exc_off = J.W.exc_off;
  int16_t *__restrict__ codes = J.W.codes;
  uint8_t *__restrict__ blob = J.blob;
  using G = Geo<NDIM>;
  using B = BoxAddr<NDIM>;
  constexpr int FAST_SIZE = FastGeo<NDIM>::ROWS * FastGeo<NDIM>::NSEG * kSegW;
  __shared__ __align__(16) int32_t box[B::SIZE > FAST_SIZE ? B::SIZE : FAST_SIZE];
  // two LDS histogram copies (even / odd lanes): escape classes put many
  // lanes of a wave on the same bin, and LDS atomics on one address serialize
  __shared__ uint32_t hist2[RECORDS ? 1 : 2 * kNSym];
  uint32_t *const hist = hist2 + (RECORDS ? 0 : (threadIdx.x & 1) * kNSym);
  __shared__ uint32_t pmask[kTilePts / 32 + 1];
  __shared__ uint32_t scr[8];

  if (dp->status != 0 || dp->is_const) return;
  if (RECORDS && !dp->big_tiles) return;  // every tile's records fit its staging slot
  const int tid = threadIdx.x;
  const float rf = dp->r_f, e2f = dp->e2_f;
  const double r = dp->r, e2 = dp->e2, eb = dp->eb;
  // float32 pre-filter bound of PatchTest<float>, rounded down; huge bounds
  // always take the exact test
  const float thr = eb < 0x1p126 ? __double2float_rd(eb * (1.0 - 0x1p-22)) : -1.0f;
  constexpr int RW = sizeof(T) / 4;  // exception records per patch
  if (!RECORDS)
    for (int s = tid; s < 2 * kNSym; s += kBlock) hist2[s] = 0;
  uint64_t my_out = 0, my_pat = 0;

  uint64_t t;
  // full tiles in the XCD-aware order; clipped tiles (the last tile row,
  // column or layer) round-robin over the workgroups, since the band order
  // would give a whole clipped tile row to one XCD
  auto next_tile = [&](uint64_t k, uint64_t *tt) -> bool {
    if (FULL) return xcd_tile(P, NDIM, k, tt, GLOBAL);
    *tt = blockIdx.x + k * gridDim.x;
    return *tt < P.n_tiles;
  };
  for (uint64_t it_k = 0; next_tile(it_k, &t); it_k++) {
    if (RECORDS && exc_cnt[t] <= (uint32_t)kStage) continue;  // uniform
    const TileGeo g = tile_geo(P, t);
    const int ez = (int)g.ez, ey = (int)g.ey, ex = (int)g.ex, nt = (int)g.nt;
    if ((nt == kTilePts) != FULL) continue;  // uniform: the other kernel's tile
    const int i0 = 32 * tid;
    int32_t d[32];
    uint32_t flags = 0;   // bit j: outlier
    uint32_t pflags = 0;  // bit j: patch
    int cnt;
    constexpr bool full = FULL;  // full tiles: residuals live in LDS, codes written
    __syncthreads();
    if (FULL) {
      // full tile: quantize into LDS, then residuals 4 points at a time
      pflags = fast_tile_load<T, NDIM, GLOBAL>(x, P, g, tid, box, rf, r, e2f, e2, eb, thr);
      __syncthreads();
      cnt = 32;
      const SegPtrs<NDIM> sp(box, tid);
      int32_t po = sp.o[-1], py = sp.y[-1], pz = sp.z[-1], pzy = sp.zy[-1];
      uint32_t run_sym = 0xffffffffu, run_n = 0;
      // The thread's 32 codes are kept (as int16 pairs) until the wave knows
      // whether all of its codes fit in int8: then they go out as bytes,
      // each lane's 32 at byte 32 * lane of the wave's 4 KiB slot (half the
      // traffic for quant's store and the encoder's two reads), else as
      // int16 at the thread's place in stream order.  Both in 16-byte
      // pieces.  int8 needs a 16-byte aligned tile start, as the encoder's
      // fast path does.
      uint32_t wq[16];
#pragma unroll
      for (int k2 = 0; k2 < 4; k2++) {
#pragma unroll
      for (int kk = 0; kk < 2; kk++) {
        const int k = 2 * k2 + kk;
        const int4 O = reinterpret_cast<const int4 *>(sp.o)[k];
        int4 Y = O, Z = O, ZY = O;
        if (NDIM >= 2) Y = reinterpret_cast<const int4 *>(sp.y)[k];
        if (NDIM == 3) {
          Z = reinterpret_cast<const int4 *>(sp.z)[k];
          ZY = reinterpret_cast<const int4 *>(sp.zy)[k];
        }
        const int32_t oa[4] = {O.x, O.y, O.z, O.w}, ya[4] = {Y.x, Y.y, Y.z, Y.w};
        const int32_t za[4] = {Z.x, Z.y, Z.z, Z.w}, zya[4] = {ZY.x, ZY.y, ZY.z, ZY.w};
        uint32_t c16[4];
        int32_t dq[4];
#pragma unroll
        for (int h = 0; h < 4; h++) {
          int32_t dv = oa[h] - po;
          if (NDIM >= 2) dv -= ya[h] - py;
          if (NDIM == 3) dv += (zya[h] - pzy) - (za[h] - pz);
          po = oa[h];
          py = ya[h];
          pz = za[h];
          pzy = zya[h];
          dq[h] = dv;
        }
        // direct symbols only (|d| <= 511 for all four points of every lane):
        // the symbol is d + 512, no escape or outlier; a wave-uniform test
        uint32_t big = 0;
#pragma unroll
        for (int h = 0; h < 4; h++) big = __builtin_elementwise_max(big, (uint32_t)(dq[h] + 511));
        const bool all_direct = !__builtin_amdgcn_ballot_w64(big > 1022u);
#pragma unroll
        for (int h = 0; h < 4; h++) {
          const int32_t dv = dq[h];
          uint32_t sy;
          if (all_direct) {
            sy = (uint32_t)(dv + 512);
            c16[h] = (uint32_t)dv & 0xffffu;
          } else {
            bool outl;
            sy = symbol_of(dv, outl);
            flags |= (outl ? 1u : 0u) << (4 * k + h);
            c16[h] = outl ? 0x8000u : ((uint32_t)dv & 0xffffu);
          }
          if (!RECORDS) {
            const bool ch = sy != run_sym;
            if (ch && run_n) atomicAdd(&hist[run_sym], run_n);
            run_n = ch ? 1u : run_n + 1u;
            run_sym = sy;
          }
        }
        wq[4 * k2 + 2 * kk] = c16[0] | (c16[1] << 16);
        wq[4 * k2 + 2 * kk + 1] = c16[2] | (c16[3] << 16);
      }
      }
      if (!RECORDS) {
        atomicAdd(&hist[run_sym], run_n);
        // int8 when every code of the wave is in -128..127 (an outlier's
        // 0x8000 is not): code + 128 in 0..255, as packed 16-bit lanes
        u16x2_t m8 = (u16x2_t)(0);
#pragma unroll
        for (int i = 0; i < 16; i++)
          m8 = __builtin_elementwise_max(m8, __builtin_bit_cast(u16x2_t, wq[i]) + (u16x2_t)(128));
        const bool w8 = (g.start & 7) == 0 && !__builtin_amdgcn_ballot_w64(m8.x > 255 || m8.y > 255);
        const int lane = tid & 63, wv = tid >> 6;
        if (lane == 0) J.W.code_w8[4 * t + wv] = w8 ? 1 : 0;
        typedef __attribute__((address_space(1))) u32x4_t gq4;
        if (w8) {
          uint32_t b[8];
#pragma unroll
          for (int m = 0; m < 8; m++) {
            const uint32_t a = wq[2 * m], c = wq[2 * m + 1];
            b[m] = (a & 0xffu) | ((a >> 8) & 0xff00u) | ((c & 0xffu) << 16) | ((c << 8) & 0xff000000u);
          }
          gq4 *dst = (gq4 *)(reinterpret_cast<uint8_t *>(codes) + 2 * g.start + 4096 * (uint64_t)wv +
                             32 * (uint64_t)lane);
          u32x4_t v0, v1;
          v0.x = b[0]; v0.y = b[1]; v0.z = b[2]; v0.w = b[3];
          v1.x = b[4]; v1.y = b[5]; v1.z = b[6]; v1.w = b[7];
          dst[0] = v0;
          dst[1] = v1;
        } else {
          gq4 *dst = (gq4 *)(codes + g.start + (uint64_t)i0);
#pragma unroll
          for (int k2 = 0; k2 < 4; k2++) {
            u32x4_t v;
            v.x = wq[4 * k2];
            v.y = wq[4 * k2 + 1];
            v.z = wq[4 * k2 + 2];
            v.w = wq[4 * k2 + 3];
            dst[k2] = v;
          }
        }
      }
    } else {
    for (int i = tid; i <= kTilePts / 32; i += kBlock) pmask[i] = 0;
    __syncthreads();

    // load phase: box rows in segments of 32 points
    constexpr int NSEG = (G::TX + 31) / 32;
    constexpr int ITEMS = B::BZ * B::BY * NSEG;
    for (int it = tid; it < ITEMS; it += kBlock) {
      const int seg = it % NSEG, row = it / NSEG;
      const int bz = row / B::BY, by = row - bz * B::BY;
      load_row<T, NDIM, GLOBAL>(x, P, g, bz, by, seg, box, pmask, rf, r, e2f, e2, eb);
    }
    __syncthreads();

    // residuals of this thread's 32 consecutive stream points
    cnt = nt - i0 < 0 ? 0 : (nt - i0 > 32 ? 32 : nt - i0);
    pflags = cnt > 0 ? ((pmask[tid]) & (cnt == 32 ? ~0u : ((1u << cnt) - 1))) : 0;
    {
      int z = 0, y = 0, xx = 0;
      if (cnt > 0) {
        z = i0 / (ey * ex);
        const int rem = i0 - z * ey * ex;
        y = rem / ex;
        xx = rem - y * ex;
      }
      // neighbours of the point before (x - 1) carried along the row
      int32_t c_prev = 0, cy_prev = 0, cz_prev = 0, cyz_prev = 0;
      bool have_prev = false;
      uint32_t run_sym = 0xffffffffu, run_n = 0;
#pragma unroll
      for (int j = 0; j < 32; j++) {
        if (j < cnt) {
          const int bz = z + G::HZ, by = y + G::HY, bx = xx + 1;
          if (!have_prev) {
            c_prev = box[B::at(bz, by, bx - 1)];
            if (NDIM >= 2) cy_prev = box[B::at(bz, by - 1, bx - 1)];
            if (NDIM == 3) { cz_prev = box[B::at(bz - 1, by, bx - 1)]; cyz_prev = box[B::at(bz - 1, by - 1, bx - 1)]; }
          }
          const int32_t c0 = box[B::at(bz, by, bx)];
          int32_t dv = c0 - c_prev;
          int32_t cy = 0, cz = 0, cyz = 0;
          if (NDIM >= 2) { cy = box[B::at(bz, by - 1, bx)]; dv += cy_prev - cy; }
          if (NDIM == 3) {
            cz = box[B::at(bz - 1, by, bx)];
            cyz = box[B::at(bz - 1, by - 1, bx)];
            dv += cyz - cz + cz_prev - cyz_prev;
          }
          c_prev = c0; cy_prev = cy; cz_prev = cz; cyz_prev = cyz;
          have_prev = true;
          d[j] = dv;
          const int32_t a = dv < 0 ? -dv : dv;
          uint32_t s;
          if (a <= 511) s = (uint32_t)(dv + 512);
          else if (a < 32768) s = 1024u + 2u * (uint32_t)(22 - __clz(a)) + (dv < 0 ? 1u : 0u);  // k - 9, k = floor(log2 a)
          else { s = 0; flags |= 1u << j; }
          if (!RECORDS) {
            if (s == run_sym) run_n++;
            else {
              if (run_n) atomicAdd(&hist[run_sym], run_n);
              run_sym = s;
              run_n = 1;
            }
          }
          if (++xx == ex) { xx = 0; have_prev = false; if (++y == ey) { y = 0; z++; } }
        }
      }
      if (!RECORDS && run_n) atomicAdd(&hist[run_sym], run_n);
    }
    }  // ragged tile
    const uint32_t nexc = __popc(flags) + RW * __popc(pflags);

    if (!RECORDS) {
      my_out += __popc(flags);
      my_pat += __popc(pflags);
    }
    if (!RECORDS && !full) {
      // residual codes, stream order
      const uint64_t base = g.start + (uint64_t)i0;
      if (cnt == 32 && (base & 7) == 0) {
        int4 *dst = reinterpret_cast<int4 *>(codes + base);
#pragma unroll
        for (int v = 0; v < 4; v++) {
          uint32_t w[4];
#pragma unroll
          for (int h = 0; h < 4; h++) {
            const int j = 8 * v + 2 * h;
            const int32_t c0 = (flags >> j) & 1u ? -32768 : d[j];
            const int32_t c1 = (flags >> (j + 1)) & 1u ? -32768 : d[j + 1];
            w[h] = ((uint32_t)c0 & 0xffffu) | ((uint32_t)c1 << 16);
          }
          dst[v] = make_int4((int)w[0], (int)w[1], (int)w[2], (int)w[3]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 32; j++)
          if (j < cnt) codes[base + j] = (int16_t)((flags >> j) & 1u ? -32768 : d[j]);
      }
    }

    // exception records in stream order: staged (or written in place by the
    // recompute pass for tiles with more than kStage records)
    uint32_t tile_total;
    const uint32_t my_off = block_excl_scan_u32(nexc, scr, &tile_total);
    if (!RECORDS && tid == 0) {
      exc_cnt[t] = tile_total;
      if (tile_total > (uint32_t)kStage) atomicOr(&dp->big_tiles, 1u);  // rare
    }
    const bool staged = tile_total <= (uint32_t)kStage;
    if (nexc && (RECORDS || staged)) {
      uint32_t e = my_off;
      const uint64_t base_off = RECORDS ? exc_off[t] : 0;
      // only the points with an outlier or a patch, in stream order
      uint32_t todo = flags | pflags;
      while (todo) {
        const int j = __ffs(todo) - 1;
        todo &= todo - 1;
        const int i = i0 + j;  // stream index inside the tile
        const int z = i / (ey * ex), rem = i - z * ey * ex;
        const int y = rem / ex, xx = rem - y * ex;
        const uint32_t pos = (uint32_t)(g.start + (uint64_t)i);
        uint32_t recs[6];
        int nr = 0;
        if ((flags >> j) & 1u) {
          recs[0] = pos;
          recs[1] = (uint32_t)(FULL ? SegPtrs<NDIM>(box, tid).d_at(j) : d[j]);
          nr = 1;
        }
        if ((pflags >> j) & 1u) {
          const uint64_t fi = ((g.z0 + z) * P.ny + (g.y0 + y)) * P.nx + (g.x0 + xx);
          uint32_t bits[2];
          const T v = x[fi];
          __builtin_memcpy(bits, &v, sizeof(T));
#pragma unroll
          for (int k = 0; k < RW; k++) { recs[2 * nr] = pos | kTagPatch; recs[2 * nr + 1] = bits[k]; nr++; }
        }
        for (int k = 0; k < nr; k++, e++) {
          if (RECORDS) {
            const uint64_t o = P.off_exc + 8 * (base_off + e);
            if (o + 8 <= P.capacity) {
              uint32_t *rec = reinterpret_cast<uint32_t *>(blob + o);
              rec[0] = recs[2 * k];
              rec[1] = recs[2 * k + 1];
            } else {
              atomicOr(&dp->overflow, 1u);
            }
          } else {
            uint32_t *rec = stage + (t * kStage + e) * 2;
            rec[0] = recs[2 * k];
            rec[1] = recs[2 * k + 1];
          }
        }
      }
    }
  }
  if (RECORDS) return;
  __syncthreads();
  for (int s = tid; s < kNSym; s += kBlock)
    if (hist2[s] + hist2[kNSym + s])
      atomicAdd(&hist_g[(blockIdx.x % kHistCopies) * kNSym + s], hist2[s] + hist2[kNSym + s]);
  my_out = wave_sum_u64(my_out);
  my_pat = wave_sum_u64(my_pat);
  if ((tid & 63) == 0) {
    if (my_out) atomicAdd((unsigned long long *)&dp->n_out, (unsigned long long)my_out);
    if (my_pat) atomicAdd((unsigned long long *)&dp->n_pat, (unsigned long long)my_pat);
  }
}

// ---------------------------------------------------------------------------
// SZ 1.4-style in-loop variant (tile domain; Sec. II-A step (1), Sec. III
// Eq. 1): a point's Lorenzo prediction reads the RECONSTRUCTED values of its
// preceding neighbours in the tile (zero outside it), the prediction error is
// quantized with bin 2 eb, and the point is reconstructed at once, so the
// next points see it.  A point whose code leaves the radius 2^15 or whose
// reconstruction misses the bound in floating point is stored exactly (the
// outlier symbol plus a patch record).  The seven prediction terms are
// summed in the field's precision in a fixed order, so that compression and
// decompression (and any other implementation that keeps the order) agree to
// the bit.  A tile is swept by diagonals: every point of diagonal
// z + y + x = d depends only on diagonals d - 1 .. d - 3, so a diagonal's
// points run in parallel, one barrier per diagonal (3D: thread (z, y) takes
// x = d - z - y; 2D: thread y takes x = d - y; 1D: one thread walks the tile).
template <typename T, int NDIM>
__device__ inline T il_pred(const T *xl, int z, int y, int x) {
  using G = Geo<NDIM>;
  auto nb = [&](int dz, int dy, int dx) -> T {
    return (z >= dz && y >= dy && x >= dx) ? xl[((z - dz) * G::TY + (y - dy)) * G::TX + (x - dx)]
                                           : (T)0;
  };
  T p = nb(0, 0, 1);
  p = p + nb(0, 1, 0);
  p = p + nb(1, 0, 0);
  p = p - nb(0, 1, 1);
  p = p - nb(1, 0, 1);
  p = p - nb(1, 1, 0);
  p = p + nb(1, 1, 1);
  return p;
}

// Runs fn(z, y, x) over the clipped tile in dependency order (all threads
// call it; it ends with a barrier).
template <int NDIM, typename Fn>
__device__ inline void il_sweep(int ez, int ey, int ex, Fn fn) {
  const int tid = threadIdx.x;
  if (NDIM == 1) {
    if (tid == 0)
      for (int x = 0; x < ex; x++) fn(0, 0, x);
    __syncthreads();
    return;
  }
  const int z = NDIM == 3 ? tid >> 4 : 0;
  const int y = NDIM == 3 ? tid & 15 : tid;
  const int nd = ez + ey + ex - 2;
  for (int d = 0; d < nd; d++) {
    const int x = d - z - y;
    if (z < ez && y < ey && x >= 0 && x < ex) fn(z, y, x);
    __syncthreads();
  }
}

template <typename T, int NDIM, bool RECORDS>
__global__ __launch_bounds__(kBlock) void k_quant_il(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const T *__restrict__ x = static_cast<const T *>(J.x);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  using G = Geo<NDIM>;
  __shared__ __align__(16) T xl[kTilePts];
  __shared__ int32_t cq[kTilePts];
  __shared__ uint32_t hist[RECORDS ? 1 : kNSym];
  __shared__ uint32_t scr[8];
  if (dp->status != 0 || dp->is_const) return;
  if (RECORDS && !dp->big_tiles) return;
  const int tid = threadIdx.x;
  const float rf = dp->r_f, e2f = dp->e2_f;
  const double r = dp->r, e2 = dp->e2, eb = dp->eb;
  constexpr int RW = sizeof(T) / 4;
  if (!RECORDS)
    for (int s = tid; s < kNSym; s += kBlock) hist[s] = 0;
  uint64_t my_pat = 0;
  uint64_t t;
  for (uint64_t it_k = 0; xcd_tile(P, NDIM, it_k, &t, false); it_k++) {
    if (RECORDS && J.W.exc_cnt[t] <= (uint32_t)kStage) continue;  // uniform
    const TileGeo g = tile_geo(P, t);
    const int ez = (int)g.ez, ey = (int)g.ey, ex = (int)g.ex, nt = (int)g.nt;
    __syncthreads();  // the previous tile's LDS is read
    for (int s = tid; s < nt; s += kBlock) {
      const int z = s / (ey * ex), rem = s - z * ey * ex, y = rem / ex, xx = rem - y * ex;
      xl[(z * G::TY + y) * G::TX + xx] =
          x[((g.z0 + z) * P.ny + (g.y0 + y)) * P.nx + (g.x0 + xx)];
    }
    __syncthreads();
    il_sweep<NDIM>(ez, ey, ex, [&](int z, int y, int xx) {
      const int i = (z * G::TY + y) * G::TX + xx;
      const T xv = xl[i];
      const T p = il_pred<T, NDIM>(xl, z, y, xx);
      const T dd = xv - p;
      int32_t q;
      T rec;
      if constexpr (sizeof(T) == 4) {
        q = (int32_t)__builtin_rintf(dd * rf);
        rec = p + (float)q * e2f;
      } else {
        q = (int32_t)__builtin_rint(dd * r);
        rec = p + (double)q * e2;
      }
      const bool keep = q > -32768 && q < 32768 && !(fabs((double)xv - (double)rec) > eb);
      xl[i] = keep ? rec : xv;
      cq[i] = keep ? q : -32768;
    });
    // this thread's 32 stream points: codes, symbols, stored points
    const int i0 = 32 * tid;
    const int cnt = nt - i0 < 0 ? 0 : (nt - i0 > 32 ? 32 : nt - i0);
    uint32_t pflags = 0;
    for (int j = 0; j < cnt; j++) {
      const int sidx = i0 + j;
      const int z = sidx / (ey * ex), rem = sidx - z * ey * ex, y = rem / ex, xx = rem - y * ex;
      const int32_t c = cq[(z * G::TY + y) * G::TX + xx];
      if (!RECORDS) {
        J.W.codes[g.start + (uint64_t)sidx] = (int16_t)c;
        bool outl;
        atomicAdd(&hist[symbol_of(c, outl)], 1u);
      }
      pflags |= (c == -32768 ? 1u : 0u) << j;
    }
    const uint32_t nexc = RW * __popc(pflags);
    if (!RECORDS) my_pat += __popc(pflags);
    uint32_t tile_total;
    const uint32_t my_off = block_excl_scan_u32(nexc, scr, &tile_total);
    if (!RECORDS && tid == 0) {
      J.W.exc_cnt[t] = tile_total;
      if (tile_total > (uint32_t)kStage) atomicOr(&dp->big_tiles, 1u);
    }
    if (nexc && (RECORDS || tile_total <= (uint32_t)kStage)) {
      uint32_t e = my_off;
      const uint64_t base_off = RECORDS ? J.W.exc_off[t] : 0;
      for (int j = 0; j < cnt; j++) {
        if (!((pflags >> j) & 1u)) continue;
        const int sidx = i0 + j;
        const int z = sidx / (ey * ex), rem = sidx - z * ey * ex, y = rem / ex, xx = rem - y * ex;
        const T v = xl[(z * G::TY + y) * G::TX + xx];  // the stored point holds x itself
        uint32_t bits[2];
        __builtin_memcpy(bits, &v, sizeof(T));
        const uint32_t key = (uint32_t)(g.start + (uint64_t)sidx) | kTagPatch;
        for (int k = 0; k < RW; k++, e++) {
          if (RECORDS) {
            const uint64_t o = P.off_exc + 8 * (base_off + e);
            if (o + 8 <= P.capacity) {
              uint32_t *rec = reinterpret_cast<uint32_t *>(J.blob + o);
              rec[0] = key;
              rec[1] = bits[k];
            } else {
              atomicOr(&dp->overflow, 1u);
            }
          } else {
            uint32_t *rec = J.W.stage + (t * kStage + e) * 2;
            rec[0] = key;
            rec[1] = bits[k];
          }
        }
      }
    }
  }
  if (RECORDS) return;
  __syncthreads();
  for (int s = tid; s < kNSym; s += kBlock)
    if (hist[s]) atomicAdd(&J.W.hist[(blockIdx.x % kHistCopies) * kNSym + s], hist[s]);
  my_pat = wave_sum_u64(my_pat);
  if ((tid & 63) == 0 && my_pat)
    atomicAdd((unsigned long long *)&dp->n_pat, (unsigned long long)my_pat);
}

// ---------------------------------------------------------------------------
// Orthogonal-transform variant (Sec. III Theorem 2, Sec. IV Theorem 3):
// blocks of 4 / 4x4 / 4x4x4 points, the orthonormal 4-point Walsh-Hadamard
// matrix H = 1/2 [[1,1,1,1], [1,1,-1,-1], [1,-1,-1,1], [1,-1,1,-1]] along x,
// then y, then z, coefficients quantized with bin 2 eb.  H is symmetric and
// H H = I, so decompression applies H again.  The sums run in the field's
// precision in the order written here (the same order wherever the scheme
// is implemented, so results agree to the bit).  Codes are in stream order:
// blocks row-major over the tile's block grid, a block's coefficients
// row-major; a block's DC bin is coded as its difference from the previous
// block's in the tile.  Each thread takes BPT consecutive blocks.
template <int NDIM> struct XfGeo;
template <> struct XfGeo<1> { static constexpr int BZ = 1, BY = 1, BS = 4, BPT = 8; };
template <> struct XfGeo<2> { static constexpr int BZ = 1, BY = 4, BS = 16, BPT = 2; };
template <> struct XfGeo<3> { static constexpr int BZ = 4, BY = 4, BS = 64, BPT = 1; };

template <typename T> __device__ inline void wht4(T &a, T &b, T &c, T &d) {
  const T w0 = ((a + b) + c) + d, w1 = ((a + b) - c) - d;
  const T w2 = ((a - b) - c) + d, w3 = ((a - b) + c) - d;
  a = (T)0.5 * w0;
  b = (T)0.5 * w1;
  c = (T)0.5 * w2;
  d = (T)0.5 * w3;
}

// a block of 4^NDIM values laid out [kz][ky][kx]
template <typename T, int NDIM> __device__ inline void wht_block(T *v) {
  constexpr int R = NDIM == 3 ? 16 : NDIM == 2 ? 4 : 1;
#pragma unroll
  for (int r = 0; r < R; r++) wht4(v[4 * r], v[4 * r + 1], v[4 * r + 2], v[4 * r + 3]);
  if (NDIM >= 2) {
#pragma unroll
    for (int kz = 0; kz < (NDIM == 3 ? 4 : 1); kz++)
#pragma unroll
      for (int kx = 0; kx < 4; kx++)
        wht4(v[16 * kz + kx], v[16 * kz + 4 + kx], v[16 * kz + 8 + kx], v[16 * kz + 12 + kx]);
  }
  if (NDIM == 3) {
#pragma unroll
    for (int r = 0; r < 16; r++) wht4(v[r], v[r + 16], v[r + 32], v[r + 48]);
  }
}

// point u of a block in the field (block origin bz0, by0, bx0 inside the tile)
template <int NDIM> __device__ inline void xf_point(int u, int &uz, int &uy, int &ux) {
  uz = NDIM == 3 ? u >> 4 : 0;
  uy = NDIM == 3 ? (u >> 2) & 3 : NDIM == 2 ? u >> 2 : 0;
  ux = u & 3;
}

template <typename T, int NDIM, bool RECORDS>
__global__ __launch_bounds__(kBlock) void k_quant_xf(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const T *__restrict__ x = static_cast<const T *>(J.x);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  using X = XfGeo<NDIM>;
  __shared__ int32_t dcs[kTilePts / 4];
  __shared__ uint32_t hist[RECORDS ? 1 : kNSym];
  __shared__ uint32_t scr[8];
  if (dp->status != 0 || dp->is_const) return;
  if (RECORDS && !dp->big_tiles) return;
  const int tid = threadIdx.x;
  const float rf = dp->r_f;
  const double r = dp->r;
  if (!RECORDS)
    for (int s = tid; s < kNSym; s += kBlock) hist[s] = 0;
  uint64_t my_out = 0;
  uint64_t t;
  for (uint64_t it_k = 0; xcd_tile(P, NDIM, it_k, &t, false); it_k++) {
    if (RECORDS && J.W.exc_cnt[t] <= (uint32_t)kStage) continue;  // uniform
    const TileGeo g = tile_geo(P, t);
    const int nbx = (int)g.ex / 4, nby = (int)g.ey / X::BY, nbz = (int)g.ez / X::BZ;
    const int nb = nbz * nby * nbx;
    __syncthreads();  // the previous tile's DC bins are read
    int32_t cq[X::BPT * X::BS];
#pragma unroll
    for (int k = 0; k < X::BPT; k++) {
      const int b = tid * X::BPT + k;
      if (b < nb) {
        const int kz = b / (nby * nbx), rem = b - kz * nby * nbx, ky = rem / nbx, kx = rem - ky * nbx;
        T v[X::BS];
#pragma unroll
        for (int u = 0; u < X::BS; u++) {
          int uz, uy, ux;
          xf_point<NDIM>(u, uz, uy, ux);
          v[u] = x[((g.z0 + (uint64_t)(kz * X::BZ + uz)) * P.ny + (g.y0 + (uint64_t)(ky * X::BY + uy))) *
                       P.nx + (g.x0 + (uint64_t)(kx * 4 + ux))];
        }
        wht_block<T, NDIM>(v);
#pragma unroll
        for (int u = 0; u < X::BS; u++) {
          if constexpr (sizeof(T) == 4) cq[k * X::BS + u] = (int32_t)__builtin_rintf(v[u] * rf);
          else cq[k * X::BS + u] = (int32_t)__builtin_rint(v[u] * r);
        }
        dcs[b] = cq[k * X::BS];
      }
    }
    __syncthreads();
    uint64_t oflags = 0;  // bit k * BS + u: outlier
#pragma unroll
    for (int k = 0; k < X::BPT; k++) {
      const int b = tid * X::BPT + k;
      if (b >= nb) continue;
      cq[k * X::BS] = (int32_t)((uint32_t)cq[k * X::BS] - (uint32_t)(b > 0 ? dcs[b - 1] : 0));
#pragma unroll
      for (int u = 0; u < X::BS; u++) {
        const int32_t c = cq[k * X::BS + u];
        bool outl;
        const uint32_t sy = symbol_of(c, outl);
        if (!RECORDS) {
          J.W.codes[g.start + (uint64_t)(b * X::BS + u)] = outl ? (int16_t)-32768 : (int16_t)c;
          atomicAdd(&hist[sy], 1u);
        }
        oflags |= (outl ? 1ull : 0ull) << (k * X::BS + u);
      }
    }
    const uint32_t nexc = (uint32_t)__popcll(oflags);
    if (!RECORDS) my_out += nexc;
    uint32_t tile_total;
    const uint32_t my_off = block_excl_scan_u32(nexc, scr, &tile_total);
    if (!RECORDS && tid == 0) {
      J.W.exc_cnt[t] = tile_total;
      if (tile_total > (uint32_t)kStage) atomicOr(&dp->big_tiles, 1u);
    }
    if (nexc && (RECORDS || tile_total <= (uint32_t)kStage)) {
      uint32_t e = my_off;
      const uint64_t base_off = RECORDS ? J.W.exc_off[t] : 0;
#pragma unroll
      for (int j = 0; j < X::BPT * X::BS; j++) {
        if (!((oflags >> j) & 1ull)) continue;
        const uint32_t pos = (uint32_t)(g.start + (uint64_t)(tid * X::BPT * X::BS + j));
        if (RECORDS) {
          const uint64_t o = P.off_exc + 8 * (base_off + e);
          if (o + 8 <= P.capacity) {
            uint32_t *rec = reinterpret_cast<uint32_t *>(J.blob + o);
            rec[0] = pos;
            rec[1] = (uint32_t)cq[j];
          } else {
            atomicOr(&dp->overflow, 1u);
          }
        } else {
          uint32_t *rec = J.W.stage + (t * kStage + e) * 2;
          rec[0] = pos;
          rec[1] = (uint32_t)cq[j];
        }
        e++;
      }
    }
  }
  if (RECORDS) return;
  __syncthreads();
  for (int s = tid; s < kNSym; s += kBlock)
    if (hist[s]) atomicAdd(&J.W.hist[(blockIdx.x % kHistCopies) * kNSym + s], hist[s]);
  my_out = wave_sum_u64(my_out);
  if ((tid & 63) == 0 && my_out)
    atomicAdd((unsigned long long *)&dp->n_out, (unsigned long long)my_out);
}

// Exclusive scan of the per-tile record counts (one workgroup): tile offsets
// into the blob's tile_exc_offset section and the workspace, the total.
constexpr int kScanThreads = 1024;
// Exclusive scan of v[0 .. n) by one workgroup of kScanThreads.  Wave w owns
// the contiguous range of R rounds of 64 elements from w R 64 (R = ceil(n /
// kScanThreads)); a round is read by the 64 lanes at once.  Pass 1 sums each
// wave's range, one block scan of the 16 wave sums follows, pass 2 scans the
// rounds in order within the wave and calls emit(k, exclusive prefix of k)
// (v[k] is read before emit, so emit may overwrite it).  Up to 16 rounds
// (n <= 16384) are all loaded at once and held in registers for pass 2;
// longer inputs keep four rounds' loads in flight and read v again in pass 2.
// Returns the total.
template <typename In, typename Emit>
__device__ inline uint64_t block_seg_scan(const In *__restrict__ v, uint64_t n, Emit emit) {
  constexpr int NW = kScanThreads / 64;
  __shared__ uint64_t wsum[NW];
  if (n == 0) return 0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint64_t R = (n + kScanThreads - 1) / kScanThreads;
  const uint64_t w0 = (uint64_t)wv * R * 64 + lane;
  auto ld = [&](uint64_t r) -> uint64_t {
    const uint64_t k = w0 + 64 * r;
    return r < R && k < n ? (uint64_t)v[k] : 0ull;
  };
  // up to kHeld rounds per wave: all loads issued at once and kept in
  // registers for pass 2
  constexpr int kHeld = 16;
  const bool held = R <= (uint64_t)kHeld;
  uint64_t xh[kHeld];
  uint64_t part = 0;
  if (held) {
    // clamped indexes: the loads issue together without branches; elements
    // past n are masked afterwards
#pragma unroll
    for (int h = 0; h < kHeld; h++) {
      const uint64_t k = w0 + 64 * (uint64_t)h;
      xh[h] = (uint64_t)v[k < n ? k : n - 1];
    }
#pragma unroll
    for (int h = 0; h < kHeld; h++) {
      xh[h] = (uint64_t)h < R && w0 + 64 * (uint64_t)h < n ? xh[h] : 0ull;
      part += xh[h];
    }
  } else {
    for (uint64_t r = 0; r < R; r += 4) {
      const uint64_t x0 = ld(r), x1 = ld(r + 1), x2 = ld(r + 2), x3 = ld(r + 3);
      part += x0 + x1 + x2 + x3;
    }
  }
  part = wave_sum_u64(part);
  if (lane == 0) wsum[wv] = part;
  __syncthreads();
  uint64_t carry = 0, tot = 0;
  for (int w = 0; w < NW; w++) {
    carry += w < wv ? wsum[w] : 0;
    tot += wsum[w];
  }
  if (held) {
#pragma unroll
    for (int h = 0; h < kHeld; h++) {
      if ((uint64_t)h >= R) break;
      const uint64_t inc = wave_incl_scan_u64(xh[h]);
      const uint64_t k = w0 + 64 * (uint64_t)h;
      if (k < n) emit(k, carry + inc - xh[h]);
      carry += __shfl(inc, 63, 64);
    }
    return tot;
  }
  for (uint64_t r = 0; r < R; r += 4) {
    uint64_t x[4];
#pragma unroll
    for (int h = 0; h < 4; h++) x[h] = ld(r + h);
#pragma unroll
    for (int h = 0; h < 4; h++) {
      const uint64_t inc = wave_incl_scan_u64(x[h]);
      const uint64_t k = w0 + 64 * (r + h);
      if (r + h < R && k < n) emit(k, carry + inc - x[h]);
      carry += __shfl(inc, 63, 64);
    }
  }
  return tot;
}

// (runs as the second workgroup of the codebook launch, beside the codebook)
__device__ inline void exc_scan_body(const CJob &J) {
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  const uint32_t *__restrict__ cnt = J.W.exc_cnt;
  uint64_t *__restrict__ off = J.W.exc_off;
  uint8_t *__restrict__ blob = J.blob;
  if (dp->status != 0 || dp->is_const) return;
  const uint64_t nt = P.n_tiles;
  uint32_t ovf = 0;
  const uint64_t tot = block_seg_scan(cnt, nt, [&](uint64_t t, uint64_t ex) {
    off[t] = ex;
    const uint64_t o = P.off_teo + 8 * t;
    if (o + 8 <= P.capacity) *reinterpret_cast<uint64_t *>(blob + o) = ex;
    else ovf = 1;
  });
  if (ovf) atomicOr(&dp->overflow, 1u);
  if (threadIdx.x == 0) {
    dp->n_exc = tot;
    dp->off_words = align8(P.off_exc + 8 * tot);
    const uint64_t o = P.off_teo + 8 * nt;
    if (o + 8 <= P.capacity) *reinterpret_cast<uint64_t *>(blob + o) = tot;
    else atomicOr(&dp->overflow, 1u);
  }
}

// ---------------------------------------------------------------------------
// a8: Huffman code lengths and canonical codes, one workgroup.
//
// The two-queue construction (leaves sorted by (count, symbol), by a rank
// sort of the nonzero bins; merged nodes in a FIFO; a leaf wins ties) is run
// in batches: with v the weight of the
// next merged node, every remaining leaf of weight <= v and every queued
// merged node is consumed before v, in merge order, so all of them can be
// ranked at once and paired.  A batch with an odd count pairs its last item
// with v itself.  The result is identical to the one-pick-at-a-time loop.
// Codes longer than 18 bits are removed by rebalancing the per-length code
// counts (two deepest siblings move up one level, one shallower code splits
// in two), and the lengths are handed out again along the (count, symbol)
// order, longest first.
constexpr int kCbThreads = 1024;

// number of entries of sorted a[0..n) that are < w (lower bound)
// Ascending sort of a[0..n) (distinct keys, n <= kSortSlots) in LDS by a
// bitonic network over the next power of two, padded with all-ones keys.
// Pair p of a stage compares slots i and i + j, i = p with a zero bit
// inserted at j; with j <= 64 a wave's pairs stay inside its own 128 slots,
// so those stages need only the wave's own LDS ordering, and a workgroup
// barrier is needed only around the stages with j >= 128.
constexpr int kSortSlots = 2048;
__device__ inline void bitonic_sort_u64(uint64_t *a, int n) {
  const int tid = threadIdx.x;
  int np2 = 2;
  while (np2 < n) np2 <<= 1;
  for (int i = n + tid; i < np2; i += (int)blockDim.x) a[i] = ~0ull;
  __syncthreads();
  for (int k = 2; k <= np2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = tid; p < (np2 >> 1); p += (int)blockDim.x) {
        const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
        const uint64_t x = a[i], y = a[i + j];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
          a[i] = y;
          a[i + j] = x;
        }
      }
      if (j >= 128 || (j == 1 && k >= 128)) {
        __syncthreads();
      } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  __syncthreads();
}

__device__ inline int count_less(const uint32_t *a, int n, uint32_t w) {
  int lo = 0, hi = n;
  while (lo < hi) { const int mid = (lo + hi) >> 1; if (a[mid] < w) lo = mid + 1; else hi = mid; }
  return lo;
}
// number of entries of sorted a[0..n) that are <= w (upper bound)
__device__ inline int count_leq(const uint32_t *a, int n, uint32_t w) {
  int lo = 0, hi = n;
  while (lo < hi) { const int mid = (lo + hi) >> 1; if (a[mid] <= w) lo = mid + 1; else hi = mid; }
  return lo;
}

// Workgroup 0 of the launch builds the code; workgroup 1 scans the tiles'
// exception counts (the two are independent).
__global__ __launch_bounds__(kCbThreads) void k_codebook(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  if (blockIdx.x == 1) {  // uniform over the block
    exc_scan_body(J);
    return;
  }
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  uint32_t *__restrict__ hist_g = J.W.hist;
  uint8_t *__restrict__ len_out = J.W.code_len;
  uint32_t *__restrict__ code_out = J.W.code;
  uint8_t *__restrict__ blob = J.blob;
  __shared__ uint64_t key[kSortSlots];  // the nonzero keys; ascending after the sort
  __shared__ uint32_t Lw[kNSym];
  __shared__ uint16_t Ls[kNSym];
  __shared__ uint32_t Iw[kNSym];
  __shared__ uint16_t parL[kNSym], parI[kNSym];
  __shared__ uint16_t dA[kNSym], pA[kNSym], dB[kNSym], pB[kNSym];
  __shared__ uint8_t lens[kNSym];
  __shared__ uint32_t lcount[kLMax + 2], lfirst[kLMax + 2], lbase[kLMax + 2];
  __shared__ uint32_t wcnt[17 * 20];
  __shared__ uint32_t bits[64];
  __shared__ int s_n, s_maxl;
  const int tid = threadIdx.x, lane = tid & 63;
  if (dp->status != 0 || dp->is_const) return;

  // nonzero bins (weight << 11 | symbol: distinct keys) in any order (one
  // slot reservation per wave), then ascending by a bitonic network
  if (tid == 0) { s_n = 0; s_maxl = 0; }
  for (int s = tid; s < kNSym; s += kCbThreads) {
    lens[s] = 0;
    Iw[s] = 0;  // merged weights are summed into place
  }
  if (tid < 64) bits[tid] = 0;
  __syncthreads();
  for (int i0 = 0; i0 < kNSym; i0 += kCbThreads) {  // uniform trip count
    const int i = i0 + tid;
    uint32_t c = 0;
    if (i < kNSym) {
#pragma unroll
      for (int k = 0; k < kHistCopies; k++) c += hist_g[k * kNSym + i];
      hist_g[i] = c;  // copy 0 keeps the total
    }
    const uint64_t m = __ballot(c != 0);
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(&s_n, __popcll(m));
    base = __shfl(base, 0, 64);
    if (c) key[base + __popcll(m & ((1ull << lane) - 1))] = ((uint64_t)c << 11) | (uint64_t)i;
  }
  __syncthreads();
  const int n = s_n;
  bitonic_sort_u64(key, n);
  if (n <= 1) {
    if (tid == 0 && n == 1) lens[key[0] & 2047] = 1;
    __syncthreads();
  } else {
    for (int j = tid; j < n; j += kCbThreads) {
      Lw[j] = (uint32_t)(key[j] >> 11);
      Ls[j] = (uint16_t)(key[j] & 2047);
    }
    __syncthreads();
    // Every thread derives a batch's bounds alike from the shared weights
    // (broadcast reads; they stay in registers), so a batch needs barriers
    // only after its ranked placement, its pairing and an odd last merge.
    // Every batch creates at least one merged node, so n - 1 batches bound
    // the loop; the guard only protects against a broken invariant.
    int li = 0, ii = 0, ni = 0;
    for (int batch = 0; batch < n; batch++) {
      if (ni >= n - 1) break;
      uint32_t w0, w1;
      {
        int a = li, c = ii;
        if (a < n && (c >= ni || Lw[a] <= Iw[c])) w0 = Lw[a++];
        else w0 = Iw[c++];
        if (a < n && (c >= ni || Lw[a] <= Iw[c])) w1 = Lw[a++];
        else w1 = Iw[c++];
      }
      const uint32_t v = w0 + w1;
      // leaves from li not heavier than v (leaf weights ascend): 64 probes
      // st apart, then the st - 1 positions after the last probe at or below
      // v (two dependent reads per wave instead of a binary search's chain)
      int ml;
      {
        const int lane = tid & 63, len = n - li, st = (len + 63) >> 6;
        const bool le1 = lane * st < len && Lw[li + lane * st] <= v;
        const int c1 = __popcll(__builtin_amdgcn_ballot_w64(le1));
        int pos = li;  // first leaf heavier than v
        if (c1 > 0) {
          const int q0 = li + (c1 - 1) * st + 1;
          const int q1 = li + c1 * st < n ? li + c1 * st : n;  // exclusive
          const bool le2 = lane < st - 1 && q0 + lane < q1 && Lw[q0 + lane] <= v;
          pos = q0 + __popcll(__builtin_amdgcn_ballot_w64(le2));
        }
        ml = pos - li;
      }
      const int nI = ni - ii, m = ml + nI;
      if (m < 2) {  // cannot happen for positive weights
        if (tid == 0) atomicOr(&dp->spin_fail, 2u);
        break;
      }
      // the items of merged rank 2p and 2p + 1 form node ni + p: each adds
      // its weight there (the slots are zero until now; integer sums do not
      // depend on the order)
      for (int k = tid; k < m; k += kCbThreads) {
        if (k < ml) {
          const uint32_t w = Lw[li + k];
          const int rank = k + count_less(Iw + ii, nI, w);
          parL[li + k] = (uint16_t)(ni + rank / 2);
          atomicAdd(&Iw[ni + rank / 2], w);
        } else {
          const int i = k - ml;
          const uint32_t w = Iw[ii + i];
          const int rank = i + count_leq(Lw + li, ml, w);
          parI[ii + i] = (uint16_t)(ni + rank / 2);
          atomicAdd(&Iw[ni + rank / 2], w);
        }
      }
      __syncthreads();
      const int half = m / 2;
      if (m & 1) {
        // the odd item (rank m - 1, already in node ni + half) pairs with
        // the lightest new node, ni
        if (tid == 0) {
          Iw[ni + half] += Iw[ni];
          parI[ni] = (uint16_t)(ni + half);
        }
        __syncthreads();
        ii = ni + 1;
        ni = ni + half + 1;
      } else {
        ii = ni;
        ni = ni + half;
      }
      li += ml;
    }
    // depths of merged nodes by pointer jumping (root = n - 2)
    const int root = n - 2;
    for (int i = tid; i < n - 1; i += kCbThreads) {
      dA[i] = i == root ? 0 : 1;
      pA[i] = i == root ? (uint16_t)root : parI[i];
    }
    __syncthreads();
    uint16_t *dc = dA, *pc = pA, *dn = dB, *pn = pB;
    for (int it = 0; it < 11; it++) {
      for (int i = tid; i < n - 1; i += kCbThreads) {
        dn[i] = (uint16_t)(dc[i] + dc[pc[i]]);
        pn[i] = pc[pc[i]];
      }
      __syncthreads();
      uint16_t *t0 = dc; dc = dn; dn = t0;
      uint16_t *t1 = pc; pc = pn; pn = t1;
    }
    // lengths, their maximum and their counts (one atomic per wave and
    // distinct length, not one per symbol on a handful of addresses)
    for (int j0 = 0; j0 < n; j0 += kCbThreads) {  // uniform trip count
      const int j = j0 + tid;
      int l = 0;
      if (j < n) {
        l = dc[parL[j]] + 1;
        l = l < 63 ? l : 63;
        lens[Ls[j]] = (uint8_t)l;
      }
      int mx = l;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
      if (lane == 0 && mx) atomicMax(&s_maxl, mx);
      uint64_t rem = __ballot(l != 0);
      while (rem) {  // uniform
        const int lv = __shfl(l, __ffsll((unsigned long long)rem) - 1, 64);
        const uint64_t mm = __ballot(l == lv);
        if (lane == 0) atomicAdd(&bits[lv], (uint32_t)__popcll(mm));
        rem &= ~mm;
      }
    }
    __syncthreads();
    if (s_maxl > kLMax) {
      // Wave 0 holds the per-length counts in registers (lane = length) and
      // computes, level by level, the state that moving one pair at a time
      // reaches.  At level i, m = bits[i] / 2 moves each put one code on
      // level i - 1 and take one split from the deepest non-empty level
      // j <= i - 2.  Those splits walk the levels 1..i-2 depth first: fully
      // using a code on level j costs 2^(i-1-j) - 1 moves and leaves
      // 2^(i-1-j) codes on level i - 1.  A suffix sum of these costs finds
      // the levels used up, the one partly used, and how far; the partly
      // used code is then split down its path.
      if (tid < 64) {
        constexpr uint64_t kSat = 1ull << 40;  // above any move count
        const int lane = tid;
        uint32_t b = bits[lane];
        const int dtop = s_maxl < 63 ? s_maxl : 63;
        bool broken = false;
        for (int i = dtop; i > kLMax; i--) {
          const uint32_t Bi = __shfl(b, i, 64);
          if (Bi & 1u) { broken = true; break; }  // not a full code tree
          const uint64_t m = Bi >> 1;
          if (lane == i) b = 0;
          if (lane == i - 1) b += (uint32_t)m;
          if (m == 0) continue;
          const bool reg = lane >= 1 && lane <= i - 2;
          const int sh = reg ? i - 1 - lane : 0;  // 1..61 inside the region
          const uint64_t cj = reg ? (1ull << sh) - 1 : 0;
          const uint64_t cs = cj < kSat ? cj : kSat;
          uint64_t T = (uint64_t)b * cs;
          T = T < kSat ? T : kSat;
          uint64_t suf = T;  // inclusive suffix sum over lanes >= lane
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            const uint64_t u = __shfl_down(suf, o, 64);
            if (lane + o < 64) suf += u;
          }
          const uint64_t total = __shfl(suf, 1, 64);
          if (total < m) { broken = true; break; }  // would split past level 1
          const uint64_t before = suf - T;
          uint64_t k = 0, r = 0;
          if (reg && before < m) {
            const uint64_t avail = m - before;
            const uint64_t q = avail / cj;
            k = q < (uint64_t)b ? q : (uint64_t)b;
            r = avail - k * cj;
          }
          const bool part = reg && before < m && k < (uint64_t)b && r > 0;
          b -= (uint32_t)k;
          const uint64_t out = wave_sum_u64(k ? (k << sh) : 0);
          if (lane == i - 1) b += (uint32_t)out;
          const uint64_t pm = __ballot(part);
          if (pm) {
            int j = __ffsll((unsigned long long)pm) - 1;
            uint64_t rr = __shfl(r, j, 64);
            while (rr > 0 && j < i - 2) {
              if (lane == j) b -= 1;
              if (lane == j + 1) b += 2;
              rr -= 1;
              j += 1;
              const uint64_t c = (1ull << (i - 1 - j)) - 1;
              if (rr >= c) {
                if (lane == j) b -= 1;
                if (lane == i - 1) b += 1u << (i - 1 - j);
                rr -= c;
              }
            }
            if (rr > 0) { broken = true; break; }
          }
        }
        bits[lane] = b;
        if (broken && lane == 0) atomicOr(&dp->spin_fail, 4u);
      }
      __syncthreads();
      // lengths re-dealt along the sorted order, longest first: position j
      // gets the longest l whose range (the counts of lengths l .. kLMax)
      // reaches past j.  The range ends are the same for every thread.
      uint32_t end[kLMax + 1];
      {
        uint32_t st = 0;
#pragma unroll
        for (int l = kLMax; l >= 1; l--) {
          st += bits[l];
          end[l] = st;
        }
      }
      for (int j = tid; j < n; j += kCbThreads) {
        int k = 0;
#pragma unroll
        for (int l = 2; l <= kLMax; l++) k += (uint32_t)j >= end[l] ? 1 : 0;
        lens[Ls[j]] = (uint8_t)(kLMax - k > 1 ? kLMax - k : 1);
      }
      __syncthreads();
    }
  }

  canonical_from_lengths(lens, code_out, lcount, lfirst, lbase, nullptr, wcnt);
  for (int s = tid; s < kNSym; s += kCbThreads) len_out[s] = lens[s];
  // code_len section (plus its 4 padding bytes)
  for (int s = tid; s < 1040; s += kCbThreads) {
    const uint64_t o = P.off_len + s;
    if (o < P.capacity) blob[o] = s < kNSym ? lens[s] : 0;
  }
}

// ---------------------------------------------------------------------------
// a9: encode.  One tile per step; bit offsets inside the tile by a block
// scan, the tile's word offset by look-back, each thread's bits packed into
// an LDS image of the tile's words and stored coalesced.

typedef __attribute__((address_space(1))) uint32_t gu32_t;
typedef __attribute__((address_space(1))) uint16_t gu16_t;

// symbol, extra-bit count and extra bits of a residual code (branch-free form
// of the symbol map)
__device__ inline uint32_t sym_ne_ev(int32_t c, uint32_t *ne, uint32_t *ev) {
  const bool outl = c == -32768;
  const int32_t a = c < 0 ? -c : c;
  const bool direct = a <= 511;
  const int k = 31 - __clz(a | 1);
  const bool esc = !direct && !outl;
  *ne = esc ? (uint32_t)k : 0u;
  *ev = esc ? (uint32_t)(a - (1 << k)) : 0u;
  const uint32_t se = 1024u + 2u * (uint32_t)(k - 9) + (c < 0 ? 1u : 0u);
  return outl ? 0u : (direct ? (uint32_t)(c + 512) : se);
}

// Encoding runs as three kernels: count (bits per thread, chunk and tile),
// an exclusive scan of the tile word counts (one workgroup per field), and
// pack.  No workgroup waits on another.  Per-thread bit counts (u16) go to
// the exception staging area, which is free once the records are placed.
struct EncCodes {
  const int16_t *codes;
  uint64_t base;
  int cnt;
  bool fast;  // 32 codes, 16-byte aligned (full tiles)
  bool w8;    // fast, and the wave's codes are stored as int8 (all direct)
  const uint8_t *bytes;    // the thread's 32 int8 codes
  u32x4_t q0, q1, q2, q3;  // the 32 codes of a fast thread, loaded up front
                           // (int8: q0, q1 hold them as bytes)
  __device__ void prefetch() {
    if (fast) {
      gptr_t<u32x4_t> src = w8 ? (gptr_t<u32x4_t>)bytes : (gptr_t<u32x4_t>)(codes + base);
      q0 = src[0];
      q1 = src[1];
      if (!w8) {
        q2 = src[2];
        q3 = src[3];
      }
    }
  }
  // fn(code + 512) for the 32 codes in order, all of them direct symbols
  // (w8, or fast with every code in -511..511)
  template <class Fn> __device__ void for_direct(Fn fn) const {
    const uint32_t w[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                            q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
    if (w8) {
#pragma unroll
      for (int i = 0; i < 8; i++)
#pragma unroll
        for (int k = 0; k < 4; k++) fn((((w[i] >> (8 * k)) & 0xffu) ^ 0x80u) + 384u);
    } else {
#pragma unroll
      for (int i = 0; i < 16; i++) {
        const u16x2_t t = __builtin_bit_cast(u16x2_t, w[i]) + (u16x2_t)(512);
        fn((uint32_t)t.x & 1023u);
        fn((uint32_t)t.y & 1023u);
      }
    }
  }
  __device__ void load8(int v, int32_t c[8]) const {
    if (fast) {
      const u32x4_t qv = v == 0 ? q0 : v == 1 ? q1 : v == 2 ? q2 : q3;
#pragma unroll
      for (int h = 0; h < 8; h++) c[h] = (int32_t)(int16_t)((qv[h >> 1] >> (16 * (h & 1))) & 0xffffu);
    } else {
#pragma unroll
      for (int h = 0; h < 8; h++) c[h] = 8 * v + h < cnt ? (int32_t)codes[base + 8 * v + h] : 0;
    }
  }
};

__device__ inline EncCodes enc_codes(const CJob &J, const TileGeo &g, uint64_t t, int tid) {
  EncCodes E;
  const int nt = (int)g.nt, i0 = 32 * tid;
  E.codes = J.W.codes;
  E.base = g.start + (uint64_t)i0;
  E.cnt = nt - i0 < 0 ? 0 : (nt - i0 > 32 ? 32 : nt - i0);
  E.fast = nt == kTilePts && (E.base & 7) == 0;  // uniform over the tile
  E.w8 = E.fast && J.W.code_w8[4 * t + (tid >> 6)] != 0;  // uniform over the wave
  E.bytes = reinterpret_cast<const uint8_t *>(J.W.codes) + 2 * g.start +
            4096 * (uint64_t)(tid >> 6) + 32 * (uint64_t)(tid & 63);
  return E;
}

__device__ inline void load_code_table(const CJob &J, uint32_t *sct) {
  for (int s = threadIdx.x; s < kNSym; s += kBlock) sct[s] = (J.W.code[s] << 8) | J.W.code_len[s];
}


// Whether every one of the 32 int16 codes of a fast thread is a direct
// symbol (residual + 512 in 1..1023).
__device__ inline bool all_direct16(const EncCodes &E) {
  const u32x4_t qs[4] = {E.q0, E.q1, E.q2, E.q3};
  u16x2_t mx = (u16x2_t)(0);
#pragma unroll
  for (int v = 0; v < 4; v++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      // (the element is copied out first: a bit cast of a vector element
      // subscript read element 0 whatever the subscript)
      const uint32_t w = qs[v][i];
      // direct: code + 511 in 0..1022 for both halves (packed 16-bit, wrapping)
      mx = __builtin_elementwise_max(mx, __builtin_bit_cast(u16x2_t, w) + (u16x2_t)(511));
    }
  return mx.x < 1023 && mx.y < 1023;
}

__global__ __launch_bounds__(kBlock) void k_enc_count(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  uint16_t *__restrict__ tb = reinterpret_cast<uint16_t *>(J.W.stage);
  uint64_t *__restrict__ tw = J.W.word_state;
  uint8_t *__restrict__ blob = J.blob;
  __shared__ uint32_t sct[kNSym];
  __shared__ uint8_t len8[1024];
  __shared__ uint32_t scr[8];
  if (dp->status != 0 || dp->is_const) return;
  const int tid = threadIdx.x;
  load_code_table(J, sct);
  for (int s = tid; s < 1024; s += kBlock) len8[s] = J.W.code_len[s];
  __syncthreads();
  for (uint64_t t = blockIdx.x; t < P.n_tiles; t += gridDim.x) {
    const TileGeo g = tile_geo(P, t);
    EncCodes E = enc_codes(J, g, t, tid);
    E.prefetch();
    // the tile's staged exception records to their place in the blob; the
    // tile's bit counts below reuse the same staging bytes, so the records
    // are read first (tiles with more records were written in place)
    {
      const uint32_t c = J.W.exc_cnt[t];  // uniform over the block
      if (c && c <= (uint32_t)kStage) {
        const uint64_t o0 = P.off_exc + 8 * J.W.exc_off[t];
        for (uint32_t e = tid; e < c; e += kBlock) {
          const uint64_t o = o0 + 8 * e;
          const uint2 v = *reinterpret_cast<const uint2 *>(J.W.stage + (t * kStage + e) * 2);
          if (o + 8 <= P.capacity) *reinterpret_cast<uint2 *>(blob + o) = v;
          else atomicOr(&dp->overflow, 1u);
        }
        __syncthreads();
      }
    }
    uint32_t bits = 0;
    bool direct = false;
    // the bits of direct symbols by one byte-table read each, when the whole
    // wave's codes are direct (the sum is not taken for a wave that needs
    // the general map below)
    if (E.fast) direct = E.w8 || all_direct16(E);
    if (!__builtin_amdgcn_ballot_w64(!direct)) E.for_direct([&](uint32_t t8) { bits += len8[t8]; });
    // the general symbol map when some lane of the wave needs it
    if (__builtin_amdgcn_ballot_w64(!direct)) {
      uint32_t gb = 0;
#pragma unroll 1
      for (int v = 0; v < 4; v++) {
        int32_t c[8];
        E.load8(v, c);
        uint32_t sy[8], ne[8], ev[8], e[8];
#pragma unroll
        for (int h = 0; h < 8; h++) sy[h] = sym_ne_ev(c[h], &ne[h], &ev[h]);
#pragma unroll
        for (int h = 0; h < 8; h++) e[h] = sct[sy[h]];
#pragma unroll
        for (int h = 0; h < 8; h++) gb += 8 * v + h < E.cnt ? (e[h] & 0xffu) + ne[h] : 0u;
      }
      bits = gb;  // every lane of the wave, direct or not
    }
    tb[t * kBlock + tid] = (uint16_t)bits;
    // chunk = 4 consecutive threads (128 symbols)
    uint32_t cb = bits;
    cb += __shfl_xor(cb, 1, 64);
    cb += __shfl_xor(cb, 2, 64);
    if ((tid & 3) == 0 && 32 * tid < (int)g.nt) {
      const uint64_t o = P.off_cb + 2 * (g.chunk_base + (uint64_t)(tid >> 2));
      if (o + 2 <= P.capacity) *(gu16_t *)(blob + o) = (uint16_t)cb;
      else atomicOr(&dp->overflow, 1u);
    }
    uint32_t tile_bits;
    (void)block_excl_scan_u32(bits, scr, &tile_bits);
    if (tid == 0) tw[t] = (tile_bits + 31) >> 5;
  }
}

__device__ inline void write_header(const CJob &J);

// exclusive scan of the tile word counts: word offsets in place, the blob's
// tile_word_offset section and the total, then the header (constant fields:
// the header only)
__global__ __launch_bounds__(kScanThreads) void k_enc_scan(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  uint64_t *__restrict__ tw = J.W.word_state;
  uint8_t *__restrict__ blob = J.blob;
  if (dp->status != 0) return;  // uniform
  if (!dp->is_const) {
    const uint64_t nt = P.n_tiles;
    uint32_t ovf = 0;
    const uint64_t tot = block_seg_scan(tw, nt, [&](uint64_t t, uint64_t ex) {
      tw[t] = ex;
      const uint64_t o = P.off_two + 8 * t;
      if (o + 8 <= P.capacity) *reinterpret_cast<uint64_t *>(blob + o) = ex;
      else ovf = 1;
    });
    if (ovf) atomicOr(&dp->overflow, 1u);
    if (threadIdx.x == 0) {
      dp->n_words = tot;
      const uint64_t o = P.off_two + 8 * nt;
      if (o + 8 <= P.capacity) *reinterpret_cast<uint64_t *>(blob + o) = tot;
      else atomicOr(&dp->overflow, 1u);
    }
  }
  __syncthreads();  // dp->n_words is visible to the workgroup
  write_header(J);
}

__global__ __launch_bounds__(kBlock) void k_enc_pack(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  const Plan P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  const uint16_t *__restrict__ tb = reinterpret_cast<const uint16_t *>(J.W.stage);
  const uint64_t *__restrict__ tw = J.W.word_state;
  uint8_t *__restrict__ blob = J.blob;
  __shared__ uint32_t words[kTilePts + 2];
  __shared__ uint32_t sct[kNSym];
  __shared__ uint32_t scr[8];
  if (dp->status != 0 || dp->is_const) return;
  const int tid = threadIdx.x;
  load_code_table(J, sct);
  const uint64_t off_words = dp->off_words;
  for (uint64_t t = blockIdx.x; t < P.n_tiles; t += gridDim.x) {
    const TileGeo g = tile_geo(P, t);
    EncCodes E = enc_codes(J, g, t, tid);
    E.prefetch();
    const uint32_t bits = tb[t * kBlock + tid];
    __syncthreads();  // previous tile's words stored; table loaded
    uint32_t tile_bits;
    const uint32_t my_bit = block_excl_scan_u32(bits, scr, &tile_bits);
    const uint32_t W = (tile_bits + 31) >> 5;
    for (uint32_t i = tid; i <= W + 1; i += kBlock) words[i] = 0;
    __syncthreads();
    // each pattern (<= 32 bits) lands in at most two words: OR both, no
    // branch; only the running bit offset links consecutive symbols
    uint32_t o = my_bit;
    auto put = [&](uint32_t pat, uint32_t pl) {
      const uint32_t w = o >> 5, b = o & 31;
      const uint64_t v = (uint64_t)pat << (64 - b - pl);
      atomicOr(&words[w], (uint32_t)(v >> 32));
      atomicOr(&words[w + 1], (uint32_t)v);
      o += pl;
    };
    // direct symbols only (residual + 512 in 1..1023, no extra bits): the
    // table entry is the whole pattern
    bool direct = E.w8;
    if (E.fast && !E.w8) {
      u16x2_t mx = (u16x2_t)(0);
      const u32x4_t qs[4] = {E.q0, E.q1, E.q2, E.q3};
#pragma unroll
      for (int v = 0; v < 4; v++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const uint32_t w = qs[v][i];  // copied out: see all_direct16
          mx = __builtin_elementwise_max(mx, __builtin_bit_cast(u16x2_t, w) + (u16x2_t)(511));
        }
      direct = mx.x < 1023 && mx.y < 1023;
    }
    if (!__builtin_amdgcn_ballot_w64(!direct)) {
      E.for_direct([&](uint32_t t8) {
        const uint32_t e = sct[t8];
        put(e >> 8, e & 0xffu);
      });
    } else {
#pragma unroll 1
      for (int v = 0; v < 4; v++) {
        int32_t c[8];
        E.load8(v, c);
        uint32_t sy[8], ne[8], ev[8], e[8];
#pragma unroll
        for (int h = 0; h < 8; h++) sy[h] = sym_ne_ev(c[h], &ne[h], &ev[h]);
#pragma unroll
        for (int h = 0; h < 8; h++) e[h] = sct[sy[h]];
        if (E.fast) {
#pragma unroll
          for (int h = 0; h < 8; h++) put(((e[h] >> 8) << ne[h]) | ev[h], (e[h] & 0xffu) + ne[h]);
        } else {
#pragma unroll
          for (int h = 0; h < 8; h++)
            if (8 * v + h < E.cnt) put(((e[h] >> 8) << ne[h]) | ev[h], (e[h] & 0xffu) + ne[h]);
        }
      }
    }
    __syncthreads();
    const uint64_t woff = tw[t];
    const uint64_t dst = off_words + 4 * woff;
    if (dst + 4ull * W <= P.capacity) {
      gu32_t *bw = (gu32_t *)(blob + dst);
      for (uint32_t i = tid; i < W; i += kBlock) bw[i] = words[i];
    } else if (tid == 0) {
      atomicOr(&dp->overflow, 1u);
    }
  }
}

// ---------------------------------------------------------------------------
// header, padding and total size (by the whole workgroup, after the word
// counts are scanned; dp->n_words written by the same workgroup)
__device__ inline void write_header(const CJob &J) {
  const Plan &P = J.P;
  DevParams *__restrict__ dp = J.W.P;
  uint8_t *__restrict__ blob = J.blob;
  const int tid = threadIdx.x;
  __shared__ uint8_t h[kHdr];
  for (int i = tid; i < (int)kHdr; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const bool cst = dp->is_const != 0;
  uint64_t total = kHdr;
  if (!cst) total = align8(dp->off_words + 4 * dp->n_words);
  if (tid == 0) {
    auto put32 = [&](int o, uint32_t v) { __builtin_memcpy(h + o, &v, 4); };
    auto put64 = [&](int o, uint64_t v) { __builtin_memcpy(h + o, &v, 8); };
    auto putf = [&](int o, double v) { __builtin_memcpy(h + o, &v, 8); };
    put32(H_MAGIC, kMagic);
    const uint16_t ver = kVersion;
    __builtin_memcpy(h + H_VERSION, &ver, 2);
    const uint16_t fl = (uint16_t)((cst ? kFlagConst : 0) | (P.domain ? kFlagTile : 0) |
                                   (P.closed ? kFlagClosed : 0) |
                                   (P.variant == kVarInloop ? kFlagInloop : 0) |
                                   (P.variant == kVarXform ? kFlagXform : 0));
    __builtin_memcpy(h + H_FLAGS, &fl, 2);
    if (P.closed) putf(H_SCALE, dp->scale);
    h[H_DTYPE] = (uint8_t)P.dtype;
    h[H_NDIM] = (uint8_t)P.ndim;
    h[H_LOG2D] = 9;
    h[H_LOG2R] = 15;
    h[H_LMAX] = kLMax;
    for (int i = 0; i < 3; i++) put64(H_DIMS + 8 * i, P.dims[i]);
    put32(H_TILE, P.tz);
    put32(H_TILE + 4, P.ty);
    put32(H_TILE + 8, P.tx);
    put32(H_CHUNK, kChunk);
    putf(H_PSNR, P.target_psnr);
    putf(H_EBREL, dp->eb_rel);
    putf(H_VR, dp->vr);
    putf(H_EB, dp->eb);
    putf(H_E2, dp->e2);
    putf(H_R, dp->r);
    if (!cst) {
      if (P.dtype == FPSZ_F32) {
        put64(H_E2T, (uint64_t)__float_as_uint(dp->e2_f));
        put64(H_RT, (uint64_t)__float_as_uint(dp->r_f));
      } else {
        put64(H_E2T, (uint64_t)__double_as_longlong(dp->e2));
        put64(H_RT, (uint64_t)__double_as_longlong(dp->r));
      }
    }
    putf(H_MIN, dp->mn);
    putf(H_MAX, dp->mx);
    put64(H_N, P.n);
    if (!cst) {
      put64(H_NTILES, P.n_tiles);
      put64(H_NCHUNKS, P.n_chunks);
      put64(H_NWORDS, dp->n_words);
      put64(H_NEXC, dp->n_exc);
      put64(H_NOUT, dp->n_out);
      put64(H_NPATCH, dp->n_pat);
    } else {
      if (P.dtype == FPSZ_F32) put64(H_CONST, (uint64_t)__float_as_uint((float)dp->mn));
      else put64(H_CONST, (uint64_t)__double_as_longlong(dp->mn));
    }
    put64(H_BYTES, total);
    dp->blob_bytes = total;
    if (total > P.capacity) dp->overflow = 1;
  }
  __syncthreads();
  for (int i = tid; i < (int)kHdr; i += blockDim.x)
    if ((uint64_t)i < P.capacity) blob[i] = h[i];
  if (!cst) {
    // zero padding after chunk_bits and after the words
    const uint64_t cb_end = P.off_cb + 2 * P.n_chunks;
    for (uint64_t o = cb_end + tid; o < align8(cb_end); o += blockDim.x)
      if (o < P.capacity) blob[o] = 0;
    const uint64_t w_end = dp->off_words + 4 * dp->n_words;
    for (uint64_t o = w_end + tid; o < align8(w_end); o += blockDim.x)
      if (o < P.capacity) blob[o] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_checksum(const uint8_t *__restrict__ blob,
                                                     uint64_t bytes_limit,
                                                     DevParams *__restrict__ dp) {
  checksum_body(blob, bytes_limit, dp, 0, blockIdx.x, gridDim.x);
}

hipError_t launch_checksum(const uint8_t *blob, uint64_t bytes, DevParams *dp, hipStream_t s) {
  const uint32_t cgrid = checksum_grid(bytes);
  hipLaunchKernelGGL(k_checksum, dim3(cgrid), dim3(kBlock), 0, s, blob, bytes, dp);
  return hipGetLastError();
}

// compress: checksum of each field's finished blob (its size from dp)
__global__ __launch_bounds__(kBlock) void k_checksum_jobs(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  checksum_body(J.blob, 0, J.W.P, 1, blockIdx.x, gridDim.x);
}

__global__ void k_checksum_store(CJob one, const CJob *__restrict__ jobs) {
  const CJob J = select_job(one, jobs);
  DevParams *__restrict__ dp = J.W.P;
  uint8_t *__restrict__ blob = J.blob;
  if (dp->status != 0 || dp->overflow) return;
  *reinterpret_cast<uint64_t *>(blob + H_CSUM) = dp->checksum;
}

// ---------------------------------------------------------------------------
LaunchCfg default_launch_cfg(const Plan &maxP) {
  LaunchCfg c;
  const uint64_t want = maxP.n / (kBlock * 16) + 1;
  // two range workgroups per CU with eight loads in flight each (measured
  // a little faster than four per CU); the autotuner may go up to kRangeBlocks
  c.range_blocks = (uint32_t)(want < (uint64_t)512 ? want : 512);
  c.quant_grid = (uint32_t)(maxP.n_tiles < 1536 ? maxP.n_tiles : 1536);
  c.encode_grid = (uint32_t)(maxP.n_tiles < 2048 ? maxP.n_tiles : 2048);
  c.csum_blocks = checksum_grid(maxP.capacity);
  return c;
}

template <typename T, int NDIM, bool GLOBAL>
static void launch_quant_d(const CJob &one, const CJob *jobs, int nf, const Plan &maxP,
                           const LaunchCfg &cfg, hipStream_t s, Timer *tm) {
  const dim3 grid(cfg.quant_grid, nf);
  if (maxP.variant == kVarXform) {
    hipLaunchKernelGGL((k_quant_xf<T, NDIM, false>), grid, dim3(kBlock), 0, s, one, jobs);
    tm->mark(s, "quant");
    hipLaunchKernelGGL(k_codebook, dim3(2, nf), dim3(kCbThreads), 0, s, one, jobs);
    tm->mark(s, "codebook");
    hipLaunchKernelGGL((k_quant_xf<T, NDIM, true>), grid, dim3(kBlock), 0, s, one, jobs);
    return;
  }
  if (maxP.variant == kVarInloop) {
    // in-loop prediction (every field of the launch; tile domain)
    hipLaunchKernelGGL((k_quant_il<T, NDIM, false>), grid, dim3(kBlock), 0, s, one, jobs);
    tm->mark(s, "quant");
    hipLaunchKernelGGL(k_codebook, dim3(2, nf), dim3(kCbThreads), 0, s, one, jobs);
    tm->mark(s, "codebook");
    hipLaunchKernelGGL((k_quant_il<T, NDIM, true>), grid, dim3(kBlock), 0, s, one, jobs);
    return;
  }
  // maxP.pad_ carries "some field of the launch has ragged tiles"
  const bool ragged = maxP.pad_ != 0;
  hipLaunchKernelGGL((k_quant<T, NDIM, GLOBAL, false, true>), grid, dim3(kBlock), 0, s, one, jobs);
  if (ragged)
    hipLaunchKernelGGL((k_quant<T, NDIM, GLOBAL, false, false>), grid, dim3(kBlock), 0, s, one, jobs);
  tm->mark(s, "quant");
  // the code and the exception offsets (one launch, two workgroups per field)
  hipLaunchKernelGGL(k_codebook, dim3(2, nf), dim3(kCbThreads), 0, s, one, jobs);
  tm->mark(s, "codebook");
  // tiles with more than kStage records recompute them in place (the others'
  // staged records are placed by the encoder's count pass)
  hipLaunchKernelGGL((k_quant<T, NDIM, GLOBAL, true, true>), grid, dim3(kBlock), 0, s, one, jobs);
  if (ragged)
    hipLaunchKernelGGL((k_quant<T, NDIM, GLOBAL, true, false>), grid, dim3(kBlock), 0, s, one, jobs);
}

template <typename T, int NDIM>
static void launch_quant(const CJob &one, const CJob *jobs, int nf, const Plan &maxP,
                         const LaunchCfg &cfg, hipStream_t s, Timer *tm) {
  if (maxP.domain == FPSZ_DOMAIN_GLOBAL)
    launch_quant_d<T, NDIM, true>(one, jobs, nf, maxP, cfg, s, tm);
  else
    launch_quant_d<T, NDIM, false>(one, jobs, nf, maxP, cfg, s, tm);
}

template <typename T>
static void launch_compress_t(const CJob &one, const CJob *jobs, int nf, const Plan &maxP,
                              const LaunchCfg &cfg, hipStream_t s, Timer *tm) {
  hipLaunchKernelGGL(k_range<T>, dim3(cfg.range_blocks, nf), dim3(kBlock), 0, s, one, jobs);
  hipLaunchKernelGGL(k_range_final, dim3(1, nf), dim3(kBlock), 0, s, one, jobs, cfg.range_blocks);
  tm->mark(s, "range");
  if (maxP.closed) {
    // the partials area holds 3 x kRangeBlocks doubles: one per k_qerr block
    hipLaunchKernelGGL(k_qerr<T>, dim3(cfg.range_blocks, nf), dim3(kBlock), 0, s, one, jobs);
    hipLaunchKernelGGL(k_rescale, dim3(1, nf), dim3(kBlock), 0, s, one, jobs, cfg.range_blocks);
    tm->mark(s, "closed_loop");
  }
  if (maxP.ndim == 1) launch_quant<T, 1>(one, jobs, nf, maxP, cfg, s, tm);
  else if (maxP.ndim == 2) launch_quant<T, 2>(one, jobs, nf, maxP, cfg, s, tm);
  else launch_quant<T, 3>(one, jobs, nf, maxP, cfg, s, tm);
  tm->mark(s, "exceptions");
  hipLaunchKernelGGL(k_enc_count, dim3(cfg.encode_grid, nf), dim3(kBlock), 0, s, one, jobs);
  hipLaunchKernelGGL(k_enc_scan, dim3(1, nf), dim3(kScanThreads), 0, s, one, jobs);
  tm->mark(s, "encode_count");
  hipLaunchKernelGGL(k_enc_pack, dim3(cfg.encode_grid, nf), dim3(kBlock), 0, s, one, jobs);
  tm->mark(s, "encode");
  hipLaunchKernelGGL(k_checksum_jobs, dim3(cfg.csum_blocks, nf), dim3(kBlock), 0, s, one, jobs);
  hipLaunchKernelGGL(k_checksum_store, dim3(1, nf), dim3(1), 0, s, one, jobs);
  tm->mark(s, "checksum");
}

// fpsz_compress_async's outcome from the field's parameter block, with the
// status rules of the synchronous call
__global__ void k_async_result(CJob one, fpsz_async_result *out) {
  if (threadIdx.x != 0) return;
  const DevParams *dp = one.W.P;
  uint32_t st = dp->status;
  if (st == 0 && dp->spin_fail) st = FPSZ_E_DEVICE;
  if (st == 0 && (dp->overflow || dp->blob_bytes > one.P.capacity)) st = FPSZ_E_CAPACITY;
  fpsz_async_result r;
  r.status = st;
  r.is_const = dp->is_const;
  r.blob_bytes = dp->blob_bytes;
  r.n_outliers = dp->n_out;
  r.n_patches = dp->n_pat;
  r.vr = dp->vr;
  r.eb = dp->eb;
  *out = r;
}

hipError_t launch_async_result(const CJob &one, fpsz_async_result *out, hipStream_t s) {
  hipLaunchKernelGGL(k_async_result, dim3(1), dim3(64), 0, s, one, out);
  return hipGetLastError();
}

hipError_t launch_compress_jobs(const CJob &one, const CJob *jobs_dev, int nf, const Plan &maxP,
                                const LaunchCfg &cfg, hipStream_t s, Timer *tm) {
  if (nf < 1 || nf > 65535 || (nf > 1 && !jobs_dev)) return hipErrorInvalidValue;
  if (!cfg.range_blocks || !cfg.quant_grid || !cfg.encode_grid || !cfg.csum_blocks)
    return hipErrorInvalidValue;
  tm->mark(s, "begin");
  if (maxP.dtype == FPSZ_F32) launch_compress_t<float>(one, jobs_dev, nf, maxP, cfg, s, tm);
  else launch_compress_t<double>(one, jobs_dev, nf, maxP, cfg, s, tm);
  return hipGetLastError();
}

}  // namespace fpsz
