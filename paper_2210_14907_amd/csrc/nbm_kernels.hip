// gfx950 kernels of the NBM training step and evaluation.
//
// Data layout in HBM (all caller-owned workspace):
//   centres      float4 [slots]           cell centres of the per-net batches
//   outputs/adj  float [slots][8]         per centre: u, du_i, eu_i (streams)
//   Zst[l]       float [tiles][S][W][16]  pre-activation streams of layer l
//   Ast[l]       op    [tiles][S][W][16]  activation streams (GEMM operands)
//   dZ           float [tiles][S][W][16]  adjoint of the pre-activations
//   partial      float [G][P]             per-work-group gradient partials
// Streams: plane 0 = base value, 1..d = first differences D_i,
// d+1..2d = second differences E_i along each axis (see nbm_device.hpp).
#include <hip/hip_runtime.h>

#include "nbm_cutcell.hpp"
#include "nbm_device.hpp"
#include "nbm_internal.hpp"
#include "nbm_launch.hpp"

namespace nbm {

// ===========================================================================
// Philox4x32-10 (Salmon et al., SC'11) and point sampling
// ===========================================================================
__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ inline int64_t range_u32(uint32_t r, uint64_t m) { return (int64_t)(((uint64_t)r * m) >> 32); }

template <int D>
__global__ void k_sample(uint64_t seed, int64_t step, int64_t jh, float* pts, int64_t n, float* bpts,
                         int64_t nb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Q = 1 << 22;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (i < n) {
    uint32_t c[4] = {(uint32_t)i, (uint32_t)step, (uint32_t)((uint64_t)step >> 32), 0u};
    philox(c, k0, k1);
    uint64_t m = (uint64_t)(2 * Q - 2 * jh + 1);
    for (int a = 0; a < D; ++a) pts[i * D + a] = (float)(range_u32(c[a], m) + jh - Q) / (float)Q;
  } else if (i < n + nb) {
    int64_t b = i - n;
    uint32_t c[4] = {(uint32_t)b, (uint32_t)step, (uint32_t)((uint64_t)step >> 32), 1u};
    philox(c, k0, k1);
    uint64_t m = (uint64_t)(2 * Q + 1);
    float x[3];
    for (int a = 0; a < D; ++a) x[a] = (float)(range_u32(c[a], m) - Q) / (float)Q;
    int face = (int)range_u32(c[3], 2 * D);
    x[face / 2] = (face % 2 == 0) ? -1.0f : 1.0f;
    for (int a = 0; a < D; ++a) bpts[b * D + a] = x[a];
  }
}

// ===========================================================================
// Classification and order-preserving compaction
// ===========================================================================
// class of an interior point: 0 = all nodes and corners in Omega^-,
// 1 = all in Omega^+, 2 = cut.  Boundary points: 0 / 1 by side.
template <int D>
__device__ inline int classify_point(const Problem& P, const float* xf, double h) {
  double x[3] = {0, 0, 0}, y[3];
  for (int a = 0; a < D; ++a) x[a] = xf[a];
  bool m0 = is_minus<D>(P, x);
  bool same = true;
  for (int a = 0; a < D && same; ++a)
    for (int sg = -1; sg <= 1; sg += 2) {
      for (int b = 0; b < D; ++b) y[b] = x[b];
      y[a] += sg * h;
      if (is_minus<D>(P, y) != m0) same = false;
    }
  for (int c = 0; c < (1 << D) && same; ++c) {
    for (int a = 0; a < D; ++a) y[a] = x[a] + h * (((c >> a) & 1) ? 0.5 : -0.5);
    if (is_minus<D>(P, y) != m0) same = false;
  }
  return same ? (m0 ? 0 : 1) : 2;
}

// coordinates of point q of the grid_n^D lattice, x_a = -1 + 2 i_a / grid_n,
// i_0 varying fastest; 32-bit division while the index fits in 32 bits (the
// 64-bit division is a long instruction sequence)
template <int D>
__device__ inline void lattice_coords(int64_t q, int grid_n, float* xf) {
  if ((uint64_t)q < (1ull << 32)) {
    uint32_t u = (uint32_t)q;
    const uint32_t gn = (uint32_t)grid_n;
    for (int a = 0; a < D; ++a) {
      const uint32_t t = u / gn;
      xf[a] = -1.0f + 2.0f * (float)(u - t * gn) / (float)grid_n;
      u = t;
    }
  } else {
    const int64_t gn = grid_n;
    for (int a = 0; a < D; ++a) { xf[a] = -1.0f + 2.0f * (float)(q % gn) / (float)gn; q /= gn; }
  }
}

// side of an evaluation point: the decision of the FP64 level set, taken from
// an FP32 evaluation of the star's phi where |phi| exceeds 1e-3 (its FP32
// rounding error is below 1e-6 for coordinates in [-1, 1] away from the
// polar axis), else from the FP64 evaluation
template <int D>
__device__ inline bool eval_minus(const Problem& P, const float* xf) {
  if (P.iface == 1) {
    const float X = xf[0], Y = xf[1], Z = D > 2 ? xf[2] : 0.0f;
    const float rho2 = X * X + Y * Y, r2 = rho2 + Z * Z;
    if (rho2 >= 1e-8f) {   // no underflow in rho^4 r^4
      const float x2 = X * X, y2 = Y * Y;
      const float im5 = Y * (5.0f * x2 * x2 - 10.0f * x2 * y2 + y2 * y2);
      const float ang = 4.0f * Z * (Z * Z - rho2) * im5 / (rho2 * rho2 * r2 * r2);
      const float ph = sqrtf(r2) - (float)P.R - (float)P.amp * ang;
      if (fabsf(ph) > 1e-3f) return ph < 0.0f;
    }
  }
  double x[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) x[a] = xf[a];
  return is_minus<D>(P, x);
}

// per-block class counts and block-local ranks (wave ballots)
// mode 0: interior points (3 classes), 1: boundary / eval points (2 sides),
// eval points are either given (pts) or generated from a grid tile.
template <int D>
__device__ inline void classify_block(const Problem& P, const float* pts, int64_t n, int mode,
                                      int64_t tile_index, int grid_n, int* cls, int* rank,
                                      int* blockcnt, int blk, int (*wcnt)[4]) {
  int64_t i = (int64_t)blk * 256 + threadIdx.x;
  int c = 3;  // 3 = no point
  if (i < n) {
    float xf[3];
    if (pts) {
      for (int a = 0; a < D; ++a) xf[a] = pts[i * D + a];
    } else {
      lattice_coords<D>(tile_index * n + i, grid_n, xf);
    }
    if (mode == 0) c = classify_point<D>(P, xf, P.h);
    else c = eval_minus<D>(P, xf) ? 0 : 1;
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int myrank = 0;
  for (int k = 0; k < 3; ++k) {
    uint64_t m = __ballot(c == k);
    if (c == k) myrank = __popcll(m & lt);
    if (lane == 0) wcnt[w][k] = __popcll(m);
  }
  __syncthreads();
  if (c < 3) {
    int off = 0;
    for (int v = 0; v < w; ++v) off += wcnt[v][c];
    cls[i] = c;
    rank[i] = off + myrank;
  }
  if (threadIdx.x < 3) {
    int s = 0;
    for (int v = 0; v < 4; ++v) s += wcnt[v][threadIdx.x];
    blockcnt[blk * 4 + threadIdx.x] = s;
  }
}

// exclusive scans of the block counts and the batch bookkeeping

// one chunk of blockDim.x consecutive entries [base, base + blockDim.x) of a
// block-count array (records of 4 ints, ncls classes used): exclusive prefix
// sums, all classes at once, by lane shuffles within each wavefront and then
// the wavefronts' totals; carry[k] enters as the offset of the chunk and
// leaves advanced by its total.  Every thread of the block calls it.
__device__ inline void scan_chunk(const int* bc, int nblk, int base, int ncls, int* off, int carry[3],
                                  int (*wsum)[4]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nws = blockDim.x / 64;
  const int idx = base + tid;
  int v[3], x[3];
  for (int k = 0; k < 3; ++k) v[k] = (idx < nblk && k < ncls) ? bc[idx * 4 + k] : 0;
  for (int k = 0; k < 3; ++k) x[k] = v[k];
  for (int d = 1; d < 64; d <<= 1)
    for (int k = 0; k < 3; ++k) {
      const int y = __shfl_up(x[k], d);
      if (lane >= d) x[k] += y;
    }
  if (lane == 63)
    for (int k = 0; k < 3; ++k) wsum[w][k] = x[k];
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    int before = 0, tot = 0;
    for (int q = 0; q < nws; ++q) {
      if (q < w) before += wsum[q][k];
      tot += wsum[q][k];
    }
    if (idx < nblk && k < ncls) off[idx * 4 + k] = carry[k] + before + x[k] - v[k];
    carry[k] += tot;
  }
  __syncthreads();
}

// first level of the scan of large batches: block g scans the g-th chunk of
// kScanThreads block counts (interior chunks, then boundary chunks) from zero
// and writes the chunk's totals, which the second level (k_scan over the
// chunk totals) turns into the chunk offsets that the scatter adds
__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(const int* bc_in, int nblk_in,
                                                              const int* bc_bnd, int nblk_bnd,
                                                              int* off_in, int* off_bnd, int* ctot_in,
                                                              int* ctot_bnd, int nchunk_in) {
  __shared__ int wsum[kScanThreads / 64][4];
  const bool bnd = (int)blockIdx.x >= nchunk_in;
  const int g = bnd ? (int)blockIdx.x - nchunk_in : (int)blockIdx.x;
  int carry[3] = {0, 0, 0};
  scan_chunk(bnd ? bc_bnd : bc_in, bnd ? nblk_bnd : nblk_in, g * kScanThreads, bnd ? 2 : 3,
             bnd ? off_bnd : off_in, carry, wsum);
  if (threadIdx.x == 0) {
    int* ct = (bnd ? ctot_bnd : ctot_in) + g * 4;
    for (int k = 0; k < 4; ++k) ct[k] = k < 3 ? carry[k] : 0;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan(const int* bc_in, int nblk_in, const int* bc_bnd,
                                              int nblk_bnd, int* off_in, int* off_bnd, Meta* meta,
                                              int n, int nb, int cut_cap, int dim, int lo,
                                              int eval_mode) {
  // exclusive prefix sums of the per-block class counts (or, for large
  // batches, of the chunk totals), 256 or kScanThreads threads
  __shared__ int wsum[kScanThreads / 64][4];
  __shared__ int totals[8];
  const int tid = threadIdx.x;
  for (int arr = 0; arr < 2; ++arr) {
    const int* bc = arr == 0 ? bc_in : bc_bnd;
    int* off = arr == 0 ? off_in : off_bnd;
    const int nblk = arr == 0 ? nblk_in : nblk_bnd;
    const int ncls = arr == 0 ? 3 : 2;
    int carry[3] = {0, 0, 0};
    for (int base = 0; base < nblk; base += (int)blockDim.x) scan_chunk(bc, nblk, base, ncls, off, carry, wsum);
    if (tid == 0)
      for (int k = 0; k < ncls; ++k) totals[arr * 4 + k] = carry[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Meta m;
    for (int a = 0; a < 2; ++a)
      for (int k = 0; k < 4; ++k) { m.cnt[a][k] = 0; m.base[a][k] = 0; }
    m.n = n;
    m.nb = nb;
    m.slow = 0;
    if (eval_mode) {
      m.ncls[0] = totals[0]; m.ncls[1] = totals[1]; m.ncls[2] = 0;
      m.nbside[0] = m.nbside[1] = 0;
      m.nB = 0; m.overflow = 0;
      m.cnt[0][KIND_A] = totals[0];
      m.cnt[1][KIND_A] = totals[1];
    } else {
      m.ncls[0] = totals[0]; m.ncls[1] = totals[1]; m.ncls[2] = totals[2];
      m.nbside[0] = totals[4]; m.nbside[1] = totals[5];
      m.overflow = totals[2] > cut_cap ? 1 : 0;
      m.nB = totals[2] < cut_cap ? totals[2] : cut_cap;
      for (int a = 0; a < 2; ++a) {
        m.cnt[a][KIND_A] = m.ncls[a];
        m.cnt[a][KIND_B] = m.nB;
        m.cnt[a][KIND_NBR] = (lo == a) ? 2 * dim * m.nB : 0;
        m.cnt[a][KIND_BND] = m.nbside[a];
      }
    }
    int tile = 0;
    for (int a = 0; a < 2; ++a) {
      int tot = 0;
      for (int k = 0; k < 4; ++k) { m.base[a][k] = tile * kTile + tot; tot += m.cnt[a][k]; }
      m.total[a] = tot;
      m.tiles[a] = (tot + kTile - 1) / kTile;
      m.tile0[a] = tile;
      tile += m.tiles[a];
    }
    *meta = m;
  }
}

// scatter: final ranks, centre lists (coordinates + source index).
// bnd = 0: interior (or evaluation) points, class < 2 -> KIND_A of that net,
// class 2 -> KIND_B of both nets (+ low-mu neighbour centres);
// bnd = 1: boundary points -> KIND_BND of the net of their side.
// one launch for both point sets: blocks [0, nblk) take the interior (or
// evaluation) points, the remaining blocks the boundary points
// operand copies W_l and W_l^T of hidden matrix m, elements 256*part ..
template <class T>
__device__ inline void shadow_block(const ShadowJobs& jobs, int m, int part) {
  const int W = jobs.W;
  const int i = part * 256 + threadIdx.x;
  if (i >= W * W) return;
  const int r = i / W, c = i % W;
  const float v = jobs.params[jobs.off[m] + i];
  ((T*)jobs.Wl[m])[i] = from_f<T>(v);
  ((T*)jobs.WlT[m])[c * W + r] = from_f<T>(v);
}

// one launch for both point sets and the operand copies: blocks [0, nblk)
// take the interior (or evaluation) points, then the boundary points up to
// nblk_cls, then `spm` blocks per hidden matrix copy the weights
template <int D>
__global__ __launch_bounds__(256) void k_classify(Problem P, const float* pts, int64_t n, int mode,
                                                  int64_t tile_index, int grid_n, int* cls, int* rank,
                                                  int* blockcnt, int nblk, const float* bpts, int64_t nb,
                                                  int* bcls, int* brank, int* blockcnt_b, int nblk_cls,
                                                  ShadowJobs jobs, int prec, int spm) {
  __shared__ int wcnt[4][4];
  const int blk = blockIdx.x;
  if (blk < nblk)
    classify_block<D>(P, pts, n, mode, tile_index, grid_n, cls, rank, blockcnt, blk, wcnt);
  else if (blk < nblk_cls)
    classify_block<D>(P, bpts, nb, 1, 0, 0, bcls, brank, blockcnt_b, blk - nblk, wcnt);
  else if (prec == 0)
    shadow_block<float>(jobs, (blk - nblk_cls) / spm, (blk - nblk_cls) % spm);
  else
    shadow_block<__bf16>(jobs, (blk - nblk_cls) / spm, (blk - nblk_cls) % spm);
}

template <int D>
__device__ inline void scatter_block(const Problem& P, const Meta* meta, const float* pts, int64_t n,
                                     const int* cls, int* rank, const int* off, const int* coff,
                                     int bnd, int64_t tile_index, int grid_n, float4* centres, int* src,
                                     int* cutidx, int blk, float* fslot) {
  int64_t i = (int64_t)blk * 256 + threadIdx.x;
  if (i >= n) return;
  int c = cls[i];
  // block offsets within their chunk, plus the chunk's offset (large batches)
  int r = rank[i] + off[blk * 4 + c] + (coff ? coff[(blk / kScanThreads) * 4 + c] : 0);
  rank[i] = r;
  float xf[3] = {0, 0, 0};
  if (pts) {
    for (int a = 0; a < D; ++a) xf[a] = pts[i * D + a];
  } else {
    lattice_coords<D>(tile_index * n + i, grid_n, xf);
  }
  float4 xc = make_float4(xf[0], xf[1], xf[2], 0.0f);
  if (bnd || c < 2) {
    int slot = meta->base[c][bnd ? KIND_BND : KIND_A] + r;
    centres[slot] = xc;
    src[slot] = (int)i;
    // manufactured forcing of an uncut point on its own side, in slot order
    if (fslot && !bnd) fslot[slot] = f_side<float, D>(P, c, xf);
    return;
  }
  if (r >= meta->nB) return;  // over capacity: dropped, the loss reports NaN
  cutidx[r] = (int)i;
  for (int a = 0; a < 2; ++a) {
    int slot = meta->base[a][KIND_B] + r;
    centres[slot] = xc;
    src[slot] = (int)i;
  }
  if (P.lo >= 0) {
    float h = (float)P.h;
    for (int k = 0; k < 2 * D; ++k) {
      float4 y = xc;
      float dv = (k & 1) ? -h : h;
      int ax = k >> 1;
      if (ax == 0) y.x += dv; else if (ax == 1) y.y += dv; else y.z += dv;
      int slot = meta->base[P.lo][KIND_NBR] + 2 * D * r + k;
      centres[slot] = y;
      src[slot] = (int)i;
    }
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_scatter(Problem P, const Meta* meta, const float* pts,
                                                 int64_t n, const int* cls, int* rank, const int* off,
                                                 int64_t tile_index, int grid_n, float4* centres,
                                                 int* src, int* cutidx, int nblk, const float* bpts,
                                                 int64_t nb, const int* bcls, int* brank,
                                                 const int* off_b, float* fslot, const int* coff,
                                                 const int* coff_b) {
  if ((int)blockIdx.x < nblk)
    scatter_block<D>(P, meta, pts, n, cls, rank, off, coff, 0, tile_index, grid_n, centres, src,
                     cutidx, blockIdx.x, fslot);
  else
    scatter_block<D>(P, meta, bpts, nb, bcls, brank, off_b, coff_b, 1, 0, 0, centres, src, cutidx,
                     blockIdx.x - nblk, nullptr);
}

// ===========================================================================
// Fourier forcing of every interior point (one thread per point).  Each
// thread keeps its phase factors exp(i pi k x_a) in LDS (rows [row][thread],
// conflict-free): row 0 holds 1 (k = 0 on any axis), rows 1..8 k_x = 1..8,
// rows 9..12 k_y = 1..4 and rows 13..16 k_z = 1..4; |k_y|, |k_z| = 5..8 are
// formed at their group's end as the factor of |k| - 4 times that of 4
// (bit 1 of the group's offset).  The modes come grouped by (k_y, k_z):
//   f = Re sum_groups e^{i pi (k_y y + k_z z)} sum_{k_x in group} c e^{i pi k_x x},
// one complex multiply-add per mode and one complex product per group; the
// mode records are read eight at a time.
// 128-thread blocks: the 17 phase rows take 17 KB of LDS per block, so nine
// blocks share a compute unit and hide the mode-record and LDS latencies.
// ===========================================================================
template <int D>
__global__ __launch_bounds__(kForcingThreads) void k_forcing(Problem P, const float* pts, int64_t n,
                                                             float* fout, const Meta* meta, const int* cls,
                                                             const int* rank, float* fslot) {
  __shared__ float2 ph[17][kForcingThreads];
  const int64_t i = (int64_t)blockIdx.x * kForcingThreads + threadIdx.x;
  const int t = threadIdx.x;
  float x[3] = {0.f, 0.f, 0.f};
  if (i < n)
    for (int a = 0; a < D; ++a) x[a] = pts[i * D + a];
  ph[0][t] = make_float2(1.f, 0.f);
  for (int a = 0; a < 3; ++a)
    for (int k = 1; k <= (a == 0 ? 8 : 4); ++k) {
      float sv, cv;
      sincospif((float)k * x[a], &sv, &cv);   // axes beyond D: x = 0, phase 1
      ph[a == 0 ? k : 4 * a + 4 + k][t] = make_float2(cv, sv);
    }
  // each thread reads only its own column: no barrier
  const char* col = reinterpret_cast<const char*>(&ph[0][t]);
  float acc = 0.0f, sre = 0.0f, sim = 0.0f;
  for (int m0 = 0; m0 < P.n_fmodes; m0 += 8) {
    // records, then their phase reads, then the arithmetic: the loads of a
    // batch are in flight together
    FMode M[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) M[u] = P.fmodes[m0 + u];
    float2 e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = *reinterpret_cast<const float2*>(col + M[u].ox);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sre += M[u].cr * e[u].x - M[u].cis * e[u].y;
      sim += M[u].ci * e[u].x + M[u].crs * e[u].y;
      if (M[u].end) {
        // close the (k_y, k_z) group: times e^{i pi (k_y y + k_z z)}
        float2 ey = *reinterpret_cast<const float2*>(col + (M[u].oy & ~3));
        float2 ez = *reinterpret_cast<const float2*>(col + (M[u].oz & ~3));
        // |k| = 5..8: times the factor of 4 (rows 12 and 16)
        auto cmul = [](float2 p, float2 q) { return make_float2(p.x * q.x - p.y * q.y, p.x * q.y + p.y * q.x); };
        if (M[u].oy & 2) ey = cmul(ey, *reinterpret_cast<const float2*>(col + 12 * kForcingThreads * 8));
        if (M[u].oz & 2) ez = cmul(ez, *reinterpret_cast<const float2*>(col + 16 * kForcingThreads * 8));
        const float yi = (M[u].oy & 1) ? -ey.y : ey.y, zi = (M[u].oz & 1) ? -ez.y : ez.y;
        const float er = ey.x * ez.x - yi * zi, ei = yi * ez.x + ey.x * zi;
        acc += sre * er - sim * ei;
        sre = 0.0f;
        sim = 0.0f;
      }
    }
  }
  if (i < n) {
    fout[i] = acc;
    // the same value in centre-slot order for uncut points (tile kernels)
    if (fslot) {
      const int c = cls[i];
      if (c < 2) fslot[meta->base[c][KIND_A] + rank[i]] = acc;
    }
  }
}

// ===========================================================================
// Utilities
// ===========================================================================
__global__ void k_fill(float* p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// grad[j] = scale * sum_g partial[g][j] in FP64: 64 columns per block, the
// G rows split over 16 groups (g = k, k+16, ...) with four running sums each;
// group sums are added in a fixed order.  With `loss`, one extra block sums
// the FP64 loss partials (fixed strided order, then a fixed tree).  Both
// outputs are NaN when the batch overflowed the cut capacity.
// Several resolution levels of one batch accumulate in FP64 across
// launches: mode 0 a single level (write grad / loss), 1 the first level
// (write the FP64 accumulators), 2 a middle level (add to them), 3 the last
// level (write accumulator + this level).
__device__ __forceinline__ double acc_level(int mode, double* slot, double v) {
  if (mode == 1) { *slot = v; return v; }
  if (mode == 2) { *slot += v; return v; }
  if (mode == 3) return *slot + v;
  return v;
}

__global__ __launch_bounds__(1024) void k_reduce(const float* partial, int G, int64_t P, float* grad,
                                                 double scale, const double* lp, int nparts,
                                                 const Meta* meta, double* loss, double* gacc,
                                                 double* lacc, int mode) {
  __shared__ double sh[16][64];
  const int c = threadIdx.x & 63, k = threadIdx.x >> 6;
  if (loss && blockIdx.x == gridDim.x - 1) {
    double* fl = &sh[0][0];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 1024) acc += lp[i];
    fl[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) fl[threadIdx.x] += fl[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double L = fl[0] / (double)(meta->n + meta->nb);
      if (meta->overflow) L = __builtin_nan("");
      L = acc_level(mode, lacc, L);
      if (mode == 0 || mode == 3) *loss = L;
    }
    return;
  }
  const int64_t j = (int64_t)blockIdx.x * 64 + c;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (j < P) {
    // 16 rows in flight per thread before any add (the adds keep a fixed
    // order), so a wave keeps 4 KB of loads outstanding
    int g = k;
    for (; g + 15 * 16 < G; g += 256) {
      float v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = partial[(int64_t)(g + 16 * u) * P + j];
#pragma unroll
      for (int u = 0; u < 16; u += 4) {
        s0 += (double)v[u];
        s1 += (double)v[u + 1];
        s2 += (double)v[u + 2];
        s3 += (double)v[u + 3];
      }
    }
    for (; g < G; g += 16) s0 += (double)partial[(int64_t)g * P + j];
  }
  sh[k][c] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (k == 0 && j < P) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += sh[q][c];
    // a batch whose cut cells overflowed the capacity dropped some of them:
    // its gradient is marked NaN like its loss, never returned partial
    double v = meta->overflow ? __builtin_nan("") : t * scale;
    v = acc_level(mode, gacc + j, v);
    if (mode == 0 || mode == 3) grad[j] = (float)v;
  }
}

__global__ __launch_bounds__(256) void k_reduce_loss(const double* lp, int nparts, const Meta* meta,
                                                     double* loss, double* lacc, int mode) {
  __shared__ double s[256];
  double acc = 0.0;
  // fixed-order strided partial sums, then a fixed tree
  for (int i = threadIdx.x; i < nparts; i += 256) acc += lp[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double L = s[0] / (double)(meta->n + meta->nb);
    if (meta->overflow) L = __builtin_nan("");
    L = acc_level(mode, lacc, L);
    if (mode == 0 || mode == 3) *loss = L;
  }
}

__global__ void k_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.0f - b1) * gi;
  float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float mh = mi / c1, vh = vi / c2;
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_counts(const Meta* meta, int* counts) {
  if (threadIdx.x == 0) {
    counts[0] = meta->ncls[0]; counts[1] = meta->ncls[1]; counts[2] = meta->ncls[2];
    counts[3] = meta->nbside[0]; counts[4] = meta->nbside[1]; counts[5] = meta->overflow;
    counts[6] = meta->slow; counts[7] = 0;
  }
}

__global__ void k_eval_out(const Meta* meta, const float* outputs, const int* src, float* u_out) {
  int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int a = 0; a < 2; ++a) {
    int64_t s0 = (int64_t)meta->tile0[a] * kTile;
    if (slot >= s0 && slot < s0 + meta->total[a]) u_out[src[slot]] = outputs[slot * 8];
  }
}

// ===========================================================================
// Block-level FP64 sum helper (fixed order)
// ===========================================================================
__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ===========================================================================
// Residual kernels (paper Sec. 3: r_p = |M^-1 A u - M^-1 b| per point)
// ===========================================================================
// uncut cells: r = -sum_i eu_i / h^2 + (k^s u - f^s(x)) / mu^s
template <int D>
__device__ inline void res_uncut_block(Problem P, const Meta* meta, const float* pts,
                                                   int64_t n, const int* cls, const int* rank,
                                                   const float* outputs, float* adj, float* resid,
                                                   double* lossp, double scale, int skip_inline,
                                                   const float* fpre, int blk) {
  __shared__ double sh[256];
  int64_t i = (int64_t)blk * 256 + threadIdx.x;
  double r2 = 0.0;
  if (i < n) {
    int c = cls[i];
    int64_t slot = c < 2 ? meta->base[c][KIND_A] + rank[i] : 0;
    if (c < 2 && skip_inline) {
      int64_t a_end = (int64_t)meta->base[c][KIND_A] + meta->cnt[c][KIND_A];
      if ((slot / kTile) * kTile + kTile <= a_end) c = 3;   // handled by the fused kernel
    }
    if (c < 2) {
      float x[3] = {0, 0, 0};
      for (int a = 0; a < D; ++a) x[a] = pts[i * D + a];
      float hh = (float)(P.h * P.h);
      float lap = 0.0f;
      for (int a = 0; a < D; ++a) lap += outputs[slot * 8 + 1 + D + a];
      float fv = fpre ? fpre[i] : f_side<float, D>(P, c, x);
      float row[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float r;
      if (P.mu_kind == 0) {
        const float kmu = (float)(P.kc[c] / P.mu[c]);
        r = -lap / hh - fv / (float)P.mu[c];
        if (kmu != 0.0f) r += kmu * outputs[slot * 8];
        const float rb = (float)(scale * (double)r);
        // the whole adjoint row (u: rb k/mu, D streams 0, E streams -rb/h^2)
        row[0] = rb * kmu;
        for (int a = 0; a < D; ++a) row[1 + D + a] = -rb / hh;
      } else {
        // mu^s at the face centres x +- (h/2) e_a (FP64: their differences
        // are O(h) and weight the O(h) first differences):
        //   R = -(1/h^2) sum_a [mu_a+ du_a + mu_a- (eu_a - du_a)] + k u - f,
        //   r = R / mubar, mubar = mean of the 2d face values
        double xd[3] = {0, 0, 0}, mup[3], mum[3], msum = 0.0;
        for (int a = 0; a < D; ++a) xd[a] = x[a];
        for (int a = 0; a < D; ++a) {
          double y[3] = {xd[0], xd[1], xd[2]};
          y[a] = xd[a] + 0.5 * P.h;
          mup[a] = mu_at<double, D>(P, c, y);
          y[a] = xd[a] - 0.5 * P.h;
          mum[a] = mu_at<double, D>(P, c, y);
          msum += mup[a] + mum[a];
        }
        const double mubar = msum / (2 * D), h2 = P.h * P.h;
        double R = P.kc[c] * (double)outputs[slot * 8] - (double)fv;
        for (int a = 0; a < D; ++a) {
          const double du = outputs[slot * 8 + 1 + a], eu = outputs[slot * 8 + 1 + D + a];
          R -= ((mup[a] - mum[a]) * du + mum[a] * eu) / h2;
        }
        r = (float)(R / mubar);
        const double rb = scale * (double)r / mubar;
        row[0] = (float)(rb * P.kc[c]);
        for (int a = 0; a < D; ++a) {
          row[1 + a] = (float)(-rb * (mup[a] - mum[a]) / h2);
          row[1 + D + a] = (float)(-rb * mum[a] / h2);
        }
      }
      if (resid) resid[i] = r;
      r2 = (double)r * (double)r;
      float4* dst = (float4*)(adj + slot * 8);
      dst[0] = make_float4(row[0], row[1], row[2], row[3]);
      dst[1] = make_float4(row[4], row[5], row[6], row[7]);
    }
  }
  double s = block_sum(r2, sh);
  if (threadIdx.x == 0) lossp[blk] = s;
}

// cut cells: full cut-cell residual in FP64 from the two networks' streams.
// One work-group of four wavefronts per cut cell, each wavefront on an
// independent piece so that the pieces run concurrently: corners / node jump
// extensions / forcing / network outputs, then face pieces / Kuhn simplices,
// then the interface term next to the flux assembly.
template <int D>
__device__ inline double res_cut_cell(Problem P, const Meta* meta, const float* pts,
                                      const int* cutidx, const float* outputs, float* adj,
                                      float* resid, double scale, const float* fpre, int blk) {
  constexpr int S = 2 * D + 1;
  constexpr int NC = 1 << D;
  constexpr int NT = D == 2 ? 2 : 6;
  __shared__ double cf[8], Jn[7], fpart[12], tvol[6], tmeas[6], tmom[6][3], os[2][7], fs[2], bt;
  __shared__ int sd[7];
  const int b = blk, tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int p = cutidx[b];
  const double h = P.h;
  double x[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) x[a] = pts[(int64_t)p * D + a];
  int64_t slot[2];
  for (int t = 0; t < 2; ++t) slot[t] = meta->base[t][KIND_B] + b;
  auto corner = [&](int c, double* q) {
    for (int a = 0; a < 3; ++a) q[a] = a < D ? x[a] + h * ((((c >> a) & 1) ? 0.5 : -0.5)) : 0.0;
  };
  // ---- phase 1
  if (wv == 0) {
    if (ln < NC) {
      double q[3];
      corner(ln, q);
      cf[ln] = phi_at<D>(P, q);
    }
  } else if (wv == 1) {
    if (ln < S) {
      const int k = ln;
      double y[3] = {x[0], x[1], x[2]};
      if (k > 0) y[(k - 1) >> 1] += ((k - 1) & 1) ? -h : h;
      sd[k] = is_minus<D>(P, y) ? 0 : 1;
      double glo[3] = {0, 0, 0};
      if (P.lo >= 0) {
        const float* ol = k == 0 ? outputs + slot[P.lo] * 8
                                 : outputs + ((int64_t)meta->base[P.lo][KIND_NBR] + 2 * D * b + (k - 1)) * 8;
        for (int a = 0; a < D; ++a) glo[a] = (2.0 * (double)ol[1 + a] - (double)ol[1 + D + a]) / (2.0 * h);
      }
      Jn[k] = jump_ext<D>(P, y, glo);
    }
  } else if (wv == 2) {
    // forcing on each side (f^- = f^+ for the Fourier forcing, precomputed)
    if (ln < 2) fs[ln] = fpre ? (double)fpre[p] : f_side<double, D>(P, ln, x);
  } else {
    if (ln < 2 * S) os[ln / S][ln % S] = outputs[slot[ln / S] * 8 + ln % S];
    // the low-mu neighbour centres (2d consecutive slots) enter through the
    // lagged normal derivative only, held fixed in the backward: zero adjoints
    if (P.lo >= 0 && ln < 2 * D * 8)
      adj[((int64_t)meta->base[P.lo][KIND_NBR] + 2 * D * b) * 8 + ln] = 0.0f;
  }
  __syncthreads();
  // ---- phase 2
  if (wv == 0) {
    if (ln < 2 * D * (D - 1)) {
      // face F, piece k: 2-D segment (k = 0), 3-D triangle k of the split square
      const int F = ln / (D - 1), k = ln % (D - 1);
      const int a = F >> 1, sgn = F & 1;
      int ids[4];
      for (int m = 0; m < (1 << (D - 1)); ++m) {
        int c = sgn == 0 ? (1 << a) : 0, t = 0;
        for (int bb = 0; bb < D; ++bb) {
          if (bb == a) continue;
          if ((m >> t) & 1) c |= 1 << bb;
          ++t;
        }
        ids[m] = c;
      }
      fpart[ln] = D == 2 ? seg_neg(cf[ids[0]], cf[ids[1]])
                         : tri_neg(cf[ids[0]], cf[ids[k == 0 ? 1 : 2]], cf[ids[3]]);
    }
  } else if (wv == 1) {
    if (ln < NT) {
      const int t = ln;
      double meas = 0.0, mom[3] = {0.0, 0.0, 0.0};
      if (D == 2) {
        const int tris[2][3] = {{0, 1, 3}, {0, 2, 3}};
        double Pt[3][3], ft[3];
        for (int i = 0; i < 3; ++i) { corner(tris[t][i], Pt[i]); ft[i] = cf[tris[t][i]]; }
        tvol[t] = tri_neg(ft[0], ft[1], ft[2]);
        iface_tri(Pt, ft, meas, mom);
      } else {
        const int tets[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
        double Pt[4][3], ft[4];
        for (int i = 0; i < 4; ++i) { corner(tets[t][i], Pt[i]); ft[i] = cf[tets[t][i]]; }
        tvol[t] = tet_neg(ft);
        iface_tet(Pt, ft, meas, mom);
      }
      tmeas[t] = meas;
      for (int a = 0; a < 3; ++a) tmom[t][a] = mom[a];
    }
  }
  __syncthreads();
  // ---- phase 3: interface term (wave 1) next to the flux assembly (wave 0)
  if (wv == 1 && ln == 0) {
    double meas = 0.0, mom[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < NT; ++t) {
      meas += tmeas[t];
      for (int a = 0; a < 3; ++a) mom[a] += tmom[t][a];
    }
    const double gamma = D == 2 ? meas / h : meas / (h * h);
    double b_t = 0.0;
    if (gamma > 0.0) {
      double cen[3], pc[3], dc, nc[3];
      for (int a = 0; a < 3; ++a) cen[a] = mom[a] / meas;
      project<D>(P, cen, pc, dc, nc);
      b_t = gamma * beta_at<D>(P, pc, nc) / h;
    }
    bt = b_t;
  }
  double vneg = 0.0, dU[6], cF[6], csum = 0.0, flux_corr = 0.0, mubar = 1.0, src = 0.0, kap = 0.0, kcorr = 0.0;
  if (tid == 0) {
    for (int t = 0; t < NT; ++t) vneg += tvol[t];
    vneg /= NT;
    // node values of the node's own network from the centre streams, and
    // U_F - U_0 from the difference streams when both nodes share a network
    for (int F = 0; F < 2 * D; ++F) {
      const int k = F + 1, a = F >> 1;
      if (sd[k] == sd[0]) {
        const int t = sd[0];
        dU[F] = (F & 1) ? os[t][1 + D + a] - os[t][1 + a] : os[t][1 + a];
      } else {
        const int t = sd[k];
        double Uk = (F & 1) ? os[t][0] + os[t][1 + D + a] - os[t][1 + a] : os[t][0] + os[t][1 + a];
        dU[F] = Uk - os[sd[0]][0];
      }
    }
    auto corr = [&](int s_, int k) -> double {
      if (s_ == 0) return sd[k] == 0 ? 0.0 : -Jn[k];
      return sd[k] == 0 ? Jn[k] : 0.0;
    };
    for (int F = 0; F < 2 * D; ++F) {
      double an = D == 2 ? fpart[F] : 0.5 * (fpart[2 * F] + fpart[2 * F + 1]);
      double ap = 1.0 - an;
      // mu^s at the face centre x +- (h/2) e_a
      double xf[3] = {x[0], x[1], x[2]};
      xf[F >> 1] += (F & 1) ? -0.5 * h : 0.5 * h;
      const double mm = mu_at<double, D>(P, 0, xf), mp = mu_at<double, D>(P, 1, xf);
      cF[F] = mm * an + mp * ap;
      csum += cF[F];
      flux_corr += mm * an * (corr(0, F + 1) - corr(0, 0)) + mp * ap * (corr(1, F + 1) - corr(1, 0));
    }
    mubar = csum / (2 * D);
    src = vneg * fs[0] + (1.0 - vneg) * fs[1];
    // Helmholtz term sum_s k^s v^s u~^s(y_0) = kap U_0 + its corrections' part
    kap = P.kc[0] * vneg + P.kc[1] * (1.0 - vneg);
    kcorr = P.kc[0] * vneg * corr(0, 0) + P.kc[1] * (1.0 - vneg) * corr(1, 0);
  }
  __syncthreads();
  if (tid != 0) return 0.0;
  const double bterm = bt;
  double R = -flux_corr / (h * h) + kcorr + kap * os[sd[0]][0] - src + bterm;
  for (int F = 0; F < 2 * D; ++F) R -= cF[F] * dU[F] / (h * h);
  double r = R / mubar;
  resid[p] = (float)r;
  // adjoints: dr/dU_F = -c_F/(h^2 mubar), dr/dU_0 = (sum_F c_F/h^2 + kap)/mubar
  double rb = scale * r;
  double Ub[7];
  Ub[0] = rb * (csum / (h * h) + kap) / mubar;
  for (int F = 0; F < 2 * D; ++F) Ub[F + 1] = -rb * cF[F] / (h * h * mubar);
  double g[2][7];
  for (int t = 0; t < 2; ++t)
    for (int s = 0; s < 7; ++s) g[t][s] = 0.0;
  for (int k = 0; k < S; ++k) {
    const int t = sd[k];
    g[t][0] += Ub[k];
    if (k > 0) {
      const int a = (k - 1) >> 1;
      if ((k - 1) & 1) { g[t][1 + D + a] += Ub[k]; g[t][1 + a] -= Ub[k]; }
      else g[t][1 + a] += Ub[k];
    }
  }
  for (int t = 0; t < 2; ++t)
    for (int s = 0; s < 8; ++s) adj[slot[t] * 8 + s] = s < S ? (float)g[t][s] : 0.0f;
  return r * r;
}

// Block blk of nblkc walks the cut cells blk, blk + nblkc, ... and writes
// their squared residuals, summed in that order, as one loss partial.
template <int D>
__device__ inline void res_cut_block(Problem P, const Meta* meta, const float* pts,
                                     const int* cutidx, const float* outputs, float* adj,
                                     float* resid, double* lossp, double scale,
                                     const float* fpre, int blk, int nblkc) {
  double acc = 0.0;
  for (int b = blk; b < meta->nB; b += nblkc) {
    acc += res_cut_cell<D>(P, meta, pts, cutidx, outputs, adj, resid, scale, fpre, b);
    __syncthreads();   // the cell's LDS scratch is rewritten by the next one
  }
  if (threadIdx.x == 0) lossp[blk] = acc;
}

// Dirichlet rows at boundary points: r_b = (2d/h^2)(u - g)
template <int D>
__device__ inline void res_bnd_block(Problem P, const Meta* meta, const float* bpts,
                                                 int64_t nb, const int* bcls, const int* brank,
                                                 const float* outputs, float* adj, float* resid,
                                                 double* lossp, double scale, int blk) {
  __shared__ double sh[256];
  int64_t i = (int64_t)blk * 256 + threadIdx.x;
  double r2 = 0.0;
  if (i < nb) {
    int c = bcls[i];
    int64_t slot = meta->base[c][KIND_BND] + brank[i];
    float x[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) x[a] = bpts[i * D + a];
    float w = (float)(2.0 * D / (P.h * P.h));
    float r = w * (outputs[slot * 8] - g_dirichlet<D>(P, x));
    resid[i] = r;
    r2 = (double)r * (double)r;
    float4* dst = (float4*)(adj + slot * 8);
    dst[0] = make_float4((float)(scale * (double)r) * w, 0.f, 0.f, 0.f);
    dst[1] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  double s = block_sum(r2, sh);
  if (threadIdx.x == 0) lossp[blk] = s;
}

// one launch for the three residual kinds: blocks [0, nblk) uncut points,
// then nblkc blocks walking the cut cells, then the boundary points
template <int D>
__global__ __launch_bounds__(256) void k_residuals(Problem P, const Meta* meta, const float* pts, int64_t n,
                                                   const int* cls, const int* rank, const int* cutidx,
                                                   const float* bpts, int64_t nb, const int* bcls,
                                                   const int* brank, const float* outputs, float* adj,
                                                   float* resid, double* lossp, double scale,
                                                   int skip_inline, const float* fpre, int nblk,
                                                   int nblkc) {
  const int blk = blockIdx.x;
  if (blk < nblk)
    res_uncut_block<D>(P, meta, pts, n, cls, rank, outputs, adj, resid, lossp, scale, skip_inline, fpre, blk);
  else if (blk < nblk + nblkc)
    res_cut_block<D>(P, meta, pts, cutidx, outputs, adj, resid, lossp + nblk, scale, fpre, blk - nblk,
                     nblkc);
  else
    res_bnd_block<D>(P, meta, bpts, nb, bcls, brank, outputs, adj, resid + n, lossp + nblk + nblkc, scale,
                     blk - nblk - nblkc);
}

// ===========================================================================
// MLP forward over difference streams (one tile of 16 centres per block)
// ===========================================================================
template <int PREC> struct Pad { static constexpr int v = PREC == 0 ? 4 : 8; };

__device__ inline int tile_net(const Meta* m, int t) {
  if (t < m->tiles[0]) return 0;
  if (t < m->tiles[0] + m->tiles[1]) return 1;
  return -1;
}

// wavefronts per block: one per 16-neuron block at W = 128 (the per-tile
// chain is the launch's critical path: its tiles are few), else four
template <int W> struct FwdWaves { static constexpr int v = W >= 128 ? 8 : 4; };

template <int D, int W, int S, int ACT, int PREC, bool STORE>
__global__ __launch_bounds__(FwdWaves<W>::v * 64) void k_forward(const Meta* meta, const float4* centres, Nets nets,
                                                 int L, float h, float* outputs, float* Zst,
                                                 void* Ast_, float* ALst, int64_t lstride,
                                                 int noninline) {
  typedef typename Op<PREC>::T T;
  constexpr int LD = W + Pad<PREC>::v;
  constexpr int NOB = W / 16;
  constexpr int KC = W / 4;  // K chunk per lane group
  constexpr int NWV = FwdWaves<W>::v, NT = 64 * NWV;
  // Row buffers, the A operand of every product.  BF16: chunk-major, the
  // 16-byte chunk k (neurons 8k .. 8k+7) of the 16 centres side by side, lane
  // group g taking chunk 4q + g at step q (one operand read = 1 KB in lane
  // order, free of LDS bank conflicts).  FP32: centre rows padded to LD.
  constexpr int kRowBuf = PREC == 1 ? kTile * W : kTile * LD;
  __shared__ __attribute__((aligned(16))) T buf[2][S][kRowBuf];
  __shared__ float part[NWV][kTile][8];
  auto rpos = [](int c, int m) {
    return PREC == 1 ? (m / 8) * (kTile * 8) + c * 8 + m % 8 : c * LD + m;
  };
  auto apos = [](int r, int gg, int q) {
    return PREC == 1 ? (4 * q + gg) * (kTile * 8) + r * 8 : r * LD + gg * KC + 4 * q;
  };
  // all tiles: one per block.  noninline: only the tiles that are not 16
  // uncut centres (the fused kernel forms the residual of those itself),
  // walked with the grid as stride: their number is known only on the
  // device, and a grid sized for the capacity would mostly churn through
  // empty blocks.
  for (int it = blockIdx.x;; it += gridDim.x) {
  int t = it;
  if (noninline) {
    int inl0 = meta->cnt[0][KIND_A] / kTile, inl1 = meta->cnt[1][KIND_A] / kTile;
    int n0 = meta->tiles[0] - inl0, n1 = meta->tiles[1] - inl1;
    if (t < n0) t = meta->tile0[0] + inl0 + t;
    else if (t < n0 + n1) t = meta->tile0[1] + inl1 + (t - n0);
    else return;
  } else if (it != (int)blockIdx.x) {
    return;
  }
  const int net = tile_net(meta, t);
  if (net < 0) return;
  const NetPtrs& np = nets.net[net];
  const int64_t slot0 = (int64_t)t * kTile;
  const int64_t slot_end = (int64_t)meta->tile0[net] * kTile + meta->total[net];
  T* Ast = (T*)Ast_;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, g = lane >> 4;

  // ---- layer 1 (K = d, VALU): z = W1 x + b1, p_i = h W1[:, i], e_i = 0
  for (int it = tid; it < kTile * W; it += NT) {
    int c = it & 15, n = it >> 4;
    float x[3] = {0, 0, 0};
    if (slot0 + c < slot_end) {
      float4 cc = centres[slot0 + c];
      x[0] = cc.x; x[1] = cc.y; x[2] = cc.z;
    }
    float z = np.b1[n];
    float p[3], e[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      float wv = np.W1[n * D + a];
      z += wv * x[a];
      p[a] = h * wv;
    }
    float av, Dv[3], Ev[3];
    if constexpr (S == 1) av = act_base<ACT>(z);
    else act_fwd<ACT, D>(z, p, e, av, Dv, Ev);
    float vals[7], pre[7];
    vals[0] = av; pre[0] = z;
    if (S > 1)
      for (int a = 0; a < D; ++a) {
        vals[1 + a] = Dv[a]; vals[1 + D + a] = Ev[a];
        pre[1 + a] = p[a]; pre[1 + D + a] = 0.0f;
      }
    for (int s = 0; s < S; ++s) {
      buf[0][s][rpos(c, n)] = from_f<T>(vals[s]);
      if (STORE) {
        int64_t o = (((int64_t)t * S + s) * W + n) * kTile + c;
        Zst[o] = pre[s];
        Ast[o] = from_f<T>(vals[s]);
      }
    }
  }
  __syncthreads();

  // ---- hidden layers 2..L on MFMA
  float vout[S][4];
  for (int s = 0; s < S; ++s)
    for (int j = 0; j < 4; ++j) vout[s][j] = 0.0f;
  // this lane's B operand (row ob*16+r16 of W_l, K chunk g; BF16: the 16-byte
  // chunks 4q + g, the row buffers' order); the first neuron block's rows of
  // the next layer are fetched one layer ahead
  struct BRow { float f[PREC == 0 ? KC : 1]; bf8 b[PREC == 1 ? KC / 8 : 1]; };
  auto load_b = [&](int l, int ob) {
    BRow r;
    const int nrow = ob * 16 + r16;
    if constexpr (PREC == 0) {
      const float4* wp = (const float4*)((const float*)np.Wl[l - 2] + (int64_t)nrow * W + g * KC);
      for (int q = 0; q < KC / 4; ++q) {
        float4 v4 = wp[q];
        r.f[4 * q] = v4.x; r.f[4 * q + 1] = v4.y; r.f[4 * q + 2] = v4.z; r.f[4 * q + 3] = v4.w;
      }
    } else {
      const bf8* wp = (const bf8*)((const T*)np.Wl[l - 2] + (int64_t)nrow * W + 8 * g);
      for (int q = 0; q < KC / 8; ++q) r.b[q] = wp[4 * q];
    }
    return r;
  };
  // (wavefronts without a neuron block, W < 16 NWV, load nothing)
  BRow bnext = w < NOB ? load_b(2, w) : BRow{};
  int cur = 0;
  for (int l = 2; l <= L; ++l) {
    const float* bl = np.bl[l - 2];
    const bool last = (l == L);
    for (int ob = w; ob < NOB; ob += NWV) {
      const int nrow = ob * 16 + r16;
      f4 acc[S];
      for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
      const BRow bcur = ob == w ? bnext : load_b(l, ob);
      if (ob + NWV >= NOB && l < L) bnext = load_b(l + 1, w);
      if constexpr (PREC == 0) {
        const float* bk = bcur.f;
        for (int s = 0; s < S; ++s) {
          const float4* ap = (const float4*)(&buf[cur][s][apos(r16, g, 0)]);
          for (int q = 0; q < KC / 4; ++q) {
            float4 a4 = ap[q];
            acc[s] = mfma4(a4.x, bk[4 * q], acc[s]);
            acc[s] = mfma4(a4.y, bk[4 * q + 1], acc[s]);
            acc[s] = mfma4(a4.z, bk[4 * q + 2], acc[s]);
            acc[s] = mfma4(a4.w, bk[4 * q + 3], acc[s]);
          }
        }
      } else {
        const bf8* bk = bcur.b;
        for (int s = 0; s < S; ++s)
          for (int q = 0; q < KC / 8; ++q)
            acc[s] = mfma32(*(const bf8*)(&buf[cur][s][apos(r16, g, q)]), bk[q], acc[s]);
      }
      // epilogue: bias, activation streams; lane holds centres 4g+j of neuron nrow
      float bias = bl[nrow];
      float wo = last ? np.wout[nrow] : 0.0f;
      for (int j = 0; j < 4; ++j) {
        float z = acc[0][j] + bias;
        float p[3], e[3], av, Dv[3], Ev[3];
        float vals[7];
        if constexpr (S == 1) {
          av = act_base<ACT>(z);
          vals[0] = av;
        } else {
          for (int a = 0; a < D; ++a) { p[a] = acc[1 + a][j]; e[a] = acc[1 + D + a][j]; }
          act_fwd<ACT, D>(z, p, e, av, Dv, Ev);
          vals[0] = av;
          for (int a = 0; a < D; ++a) { vals[1 + a] = Dv[a]; vals[1 + D + a] = Ev[a]; }
        }
        acc[0][j] = z;
        for (int s = 0; s < S; ++s) {
          if (!last) buf[cur ^ 1][s][rpos(4 * g + j, nrow)] = from_f<T>(vals[s]);
          else vout[s][j] += wo * vals[s];
        }
        if (STORE) {
          for (int s = 0; s < S; ++s) {
            int64_t o = (((int64_t)t * S + s) * W + nrow) * kTile + 4 * g + j;
            if (!last) Ast[(int64_t)(l - 1) * lstride + o] = from_f<T>(vals[s]);
            else ALst[o] = vals[s];
          }
        }
      }
      if (STORE) {
        for (int s = 0; s < S; ++s) {
          int64_t o = (((int64_t)t * S + s) * W + nrow) * kTile + 4 * g;
          float4 zv = make_float4(acc[s][0], acc[s][1], acc[s][2], acc[s][3]);
          *(float4*)(Zst + (int64_t)(l - 1) * lstride + o) = zv;
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  // ---- output layer: u = w_out . a + b_out, du_i = w_out . D_i, eu_i = w_out . E_i
  for (int s = 0; s < S; ++s)
    for (int j = 0; j < 4; ++j) {
      float v = vout[s][j];
      v += __shfl_xor(v, 8);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 1);
      vout[s][j] = v;
    }
  if (r16 == 0)
    for (int s = 0; s < S; ++s)
      for (int j = 0; j < 4; ++j) part[w][4 * g + j][s] = vout[s][j];
  __syncthreads();
  if (tid < kTile * S) {
    int c = tid / S, s = tid % S;
    float v = part[0][c][s];
    for (int q = 1; q < NWV; ++q) v += part[q][c][s];
    if (s == 0) v += np.bout[0];
    if (slot0 + c < slot_end) outputs[(slot0 + c) * 8 + s] = v;
  }
  __syncthreads();   // part is rewritten by the next tile
  }
}

// ===========================================================================
// MLP backward for hidden layer l (persistent work-groups; each accumulates
// dW_l over its tiles in MFMA accumulators and writes one partial row)
// ===========================================================================
template <int D, int W, int ACT, int PREC>
__global__ __launch_bounds__(256) void k_backward(const Meta* meta, const float4* centres, Nets nets,
                                                  int L, int l, float h, const float* adj,
                                                  const float* Zst, const void* Ast_,
                                                  const float* ALst, float* dZ, float* partial,
                                                  int64_t Ptot, NetLayout lay, int64_t net_off1,
                                                  int64_t lstride) {
  typedef typename Op<PREC>::T T;
  constexpr int S = 2 * D + 1;
  constexpr int LD = W + Pad<PREC>::v;
  constexpr int NOB = W / 16;
  constexpr int OBW = (NOB + 3) / 4;
  constexpr int KC = W / 4;
  __shared__ __attribute__((aligned(16))) T dzrow[S][kTile][LD];
  __shared__ float adjs[kTile][8];
  __shared__ float xs[kTile][4];
  const T* Ast = (const T*)Ast_;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, g = lane >> 4;
  const int G = gridDim.x;
  const int ntiles = meta->tiles[0] + meta->tiles[1];
  const bool top = (l == L), bottom = (l == 2);

  for (int net = 0; net < 2; ++net) {
    const NetPtrs& np = nets.net[net];
    const T* WmT = (const T*)np.WlT[l - 2];
    f4 accW[OBW][NOB];
    float accb[OBW], accwo[OBW], accW1[OBW][3], accb1[OBW];
    float accbo = 0.0f;
    for (int i = 0; i < OBW; ++i) {
      for (int k = 0; k < NOB; ++k) accW[i][k] = f4{0.f, 0.f, 0.f, 0.f};
      accb[i] = 0.f; accwo[i] = 0.f; accb1[i] = 0.f;
      for (int a = 0; a < 3; ++a) accW1[i][a] = 0.f;
    }
    for (int t = blockIdx.x; t < ntiles; t += G) {
      if (tile_net(meta, t) != net) continue;
      const int64_t slot0 = (int64_t)t * kTile;
      if (tid < kTile * 8) {
        int c = tid >> 3, s = tid & 7;
        adjs[c][s] = top ? adj[(slot0 + c) * 8 + s] : 0.0f;
      }
      if (tid < kTile) {
        float4 cc = centres[slot0 + tid];
        const int64_t slot_end = (int64_t)meta->tile0[net] * kTile + meta->total[net];
        if (slot0 + tid >= slot_end) cc = make_float4(0.f, 0.f, 0.f, 0.f);
        xs[tid][0] = cc.x; xs[tid][1] = cc.y; xs[tid][2] = cc.z; xs[tid][3] = 0.f;
      }
      __syncthreads();
      // ---- dZ_l for the out-blocks owned by this wave (accumulator layout)
      float dz[OBW][S][4];
      for (int i = 0; i < OBW; ++i) {
        int ob = w + 4 * i;
        if (ob >= NOB) break;
        int n = ob * 16 + r16;
        if (top) {
          float wo = np.wout[n];
          for (int s = 0; s < S; ++s) {
            int64_t o = (((int64_t)t * S + s) * W + n) * kTile + 4 * g;
            float4 zv = *(const float4*)(Zst + (int64_t)(l - 1) * lstride + o);
            float4 av = *(const float4*)(ALst + o);
            float za[4] = {zv.x, zv.y, zv.z, zv.w}, aa[4] = {av.x, av.y, av.z, av.w};
            for (int j = 0; j < 4; ++j) {
              dz[i][s][j] = za[j];
              accwo[i] += adjs[4 * g + j][s] * aa[j];
            }
          }
          for (int j = 0; j < 4; ++j) {
            float p[3], e[3], Db[3], Eb[3], zb, pb[3], eb[3];
            for (int a = 0; a < D; ++a) {
              p[a] = dz[i][1 + a][j]; e[a] = dz[i][1 + D + a][j];
              Db[a] = wo * adjs[4 * g + j][1 + a]; Eb[a] = wo * adjs[4 * g + j][1 + D + a];
            }
            act_bwd<ACT, D>(dz[i][0][j], p, e, wo * adjs[4 * g + j][0], Db, Eb, zb, pb, eb);
            dz[i][0][j] = zb;
            for (int a = 0; a < D; ++a) { dz[i][1 + a][j] = pb[a]; dz[i][1 + D + a][j] = eb[a]; }
          }
        } else {
          for (int s = 0; s < S; ++s) {
            int64_t o = (((int64_t)t * S + s) * W + n) * kTile + 4 * g;
            float4 v = *(const float4*)(dZ + o);
            dz[i][s][0] = v.x; dz[i][s][1] = v.y; dz[i][s][2] = v.z; dz[i][s][3] = v.w;
          }
        }
        for (int j = 0; j < 4; ++j) accb[i] += dz[i][0][j];
      }
      if (top && tid == 0)
        for (int c = 0; c < kTile; ++c) accbo += adjs[c][0];
      // ---- dW_l += dZ_l^T A_{l-1}: K runs over (stream, centre)
      for (int ib = 0; ib < NOB; ++ib) {
        const int nin = ib * 16 + r16;
        if constexpr (PREC == 0) {
          float ap[S][4];
          for (int s = 0; s < S; ++s) {
            int64_t o = (((int64_t)t * S + s) * W + nin) * kTile + 4 * g;
            float4 v = *(const float4*)((const float*)Ast + (int64_t)(l - 2) * lstride + o);
            ap[s][0] = v.x; ap[s][1] = v.y; ap[s][2] = v.z; ap[s][3] = v.w;
          }
          for (int i = 0; i < OBW; ++i) {
            if (w + 4 * i >= NOB) break;
            for (int s = 0; s < S; ++s)
              for (int j = 0; j < 4; ++j) accW[i][ib] = mfma4(dz[i][s][j], ap[s][j], accW[i][ib]);
          }
        } else {
          bf4 ap[S + 1];
          for (int s = 0; s < S; ++s) {
            int64_t o = (((int64_t)t * S + s) * W + nin) * kTile + 4 * g;
            ap[s] = *(const bf4*)(Ast + (int64_t)(l - 2) * lstride + o);
          }
          ap[S] = bf4{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
          for (int i = 0; i < OBW; ++i) {
            if (w + 4 * i >= NOB) break;
            for (int s = 0; s < S; s += 2) {
              bf8 av, bv;
              for (int j = 0; j < 4; ++j) {
                av[j] = (__bf16)dz[i][s][j];
                av[4 + j] = (s + 1 < S) ? (__bf16)dz[i][s + 1][j] : (__bf16)0.f;
                bv[j] = ap[s][j];
                bv[4 + j] = ap[s + 1][j];
              }
              accW[i][ib] = mfma32(av, bv, accW[i][ib]);
            }
          }
        }
      }
      // ---- dA: abar_{l-1} = dZ_l W_l, then dZ_{l-1} from the stored pre-activations
      for (int i = 0; i < OBW; ++i) {
        int ob = w + 4 * i;
        if (ob >= NOB) break;
        for (int s = 0; s < S; ++s)
          for (int j = 0; j < 4; ++j) dzrow[s][4 * g + j][ob * 16 + r16] = from_f<T>(dz[i][s][j]);
      }
      __syncthreads();
      for (int i = 0; i < OBW; ++i) {
        int ib = w + 4 * i;
        if (ib >= NOB) break;
        const int nin = ib * 16 + r16;
        f4 acc[S];
        for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == 0) {
          float bk[KC];
          const float4* wp = (const float4*)((const float*)WmT + (int64_t)nin * W + g * KC);
          for (int q = 0; q < KC / 4; ++q) {
            float4 v4 = wp[q];
            bk[4 * q] = v4.x; bk[4 * q + 1] = v4.y; bk[4 * q + 2] = v4.z; bk[4 * q + 3] = v4.w;
          }
          for (int s = 0; s < S; ++s) {
            const float4* ap = (const float4*)(&dzrow[s][r16][g * KC]);
            for (int q = 0; q < KC / 4; ++q) {
              float4 a4 = ap[q];
              acc[s] = mfma4(a4.x, bk[4 * q], acc[s]);
              acc[s] = mfma4(a4.y, bk[4 * q + 1], acc[s]);
              acc[s] = mfma4(a4.z, bk[4 * q + 2], acc[s]);
              acc[s] = mfma4(a4.w, bk[4 * q + 3], acc[s]);
            }
          }
        } else {
          bf8 bk[KC / 8];
          const bf8* wp = (const bf8*)((const T*)WmT + (int64_t)nin * W + g * KC);
          for (int q = 0; q < KC / 8; ++q) bk[q] = wp[q];
          for (int s = 0; s < S; ++s) {
            const bf8* ap = (const bf8*)(&dzrow[s][r16][g * KC]);
            for (int q = 0; q < KC / 8; ++q) acc[s] = mfma32(ap[q], bk[q], acc[s]);
          }
        }
        // pre-activations of layer l-1
        float zp[S][4];
        for (int s = 0; s < S; ++s) {
          int64_t o = (((int64_t)t * S + s) * W + nin) * kTile + 4 * g;
          float4 v = *(const float4*)(Zst + (int64_t)(l - 2) * lstride + o);
          zp[s][0] = v.x; zp[s][1] = v.y; zp[s][2] = v.z; zp[s][3] = v.w;
        }
        float out[S][4];
        for (int j = 0; j < 4; ++j) {
          float p[3], e[3], Db[3], Eb[3], zb, pb[3], eb[3];
          for (int a = 0; a < D; ++a) {
            p[a] = zp[1 + a][j]; e[a] = zp[1 + D + a][j];
            Db[a] = acc[1 + a][j]; Eb[a] = acc[1 + D + a][j];
          }
          act_bwd<ACT, D>(zp[0][j], p, e, acc[0][j], Db, Eb, zb, pb, eb);
          out[0][j] = zb;
          for (int a = 0; a < D; ++a) { out[1 + a][j] = pb[a]; out[1 + D + a][j] = eb[a]; }
        }
        if (!bottom) {
          for (int s = 0; s < S; ++s) {
            int64_t o = (((int64_t)t * S + s) * W + nin) * kTile + 4 * g;
            *(float4*)(dZ + o) = make_float4(out[s][0], out[s][1], out[s][2], out[s][3]);
          }
        } else {
          // layer 1: z = W1 x + b1, p_a = h W1[:, a]
          for (int j = 0; j < 4; ++j) {
            int c = 4 * g + j;
            accb1[i] += out[0][j];
            for (int a = 0; a < D; ++a) accW1[i][a] += out[0][j] * xs[c][a] + h * out[1 + a][j];
          }
        }
      }
      __syncthreads();
    }
    // ---- flush this net's partial gradient
    float* prow = partial + (int64_t)blockIdx.x * Ptot + (net == 0 ? 0 : net_off1);
    for (int i = 0; i < OBW; ++i) {
      int ob = w + 4 * i;
      if (ob >= NOB) break;
      for (int ib = 0; ib < NOB; ++ib)
        for (int r = 0; r < 4; ++r) {
          int row = ob * 16 + 4 * g + r, col = ib * 16 + r16;
          prow[lay.Wl[l - 2] + (int64_t)row * W + col] = accW[i][ib][r];
        }
      float vb = accb[i];
      vb += __shfl_xor(vb, 16);
      vb += __shfl_xor(vb, 32);
      float vwo = accwo[i];
      vwo += __shfl_xor(vwo, 16);
      vwo += __shfl_xor(vwo, 32);
      float vb1 = accb1[i], vw1[3];
      vb1 += __shfl_xor(vb1, 16);
      vb1 += __shfl_xor(vb1, 32);
      for (int a = 0; a < 3; ++a) {
        vw1[a] = accW1[i][a];
        vw1[a] += __shfl_xor(vw1[a], 16);
        vw1[a] += __shfl_xor(vw1[a], 32);
      }
      int n = ob * 16 + r16;
      if (g == 0) {
        prow[lay.bl[l - 2] + n] = vb;
        if (top) prow[lay.wout + n] = vwo;
        if (bottom) {
          prow[lay.b1 + n] = vb1;
          for (int a = 0; a < D; ++a) prow[lay.W1 + (int64_t)n * D + a] = vw1[a];
        }
      }
    }
    if (top && tid == 0) prow[lay.bout] = accbo;
  }
}

// ===========================================================================
// Host-side launchers
// ===========================================================================
template <int D, int W, int ACT, int PREC>
struct Launch {
  static hipError_t forward(hipStream_t st, int grid, const Meta* meta, const float4* centres,
                            const Nets& nets, int L, float h, float* outputs, float* Zst, void* Ast,
                            float* ALst, int64_t lstride, bool store, bool streams, int noninline) {
    if (streams && store)
      hipLaunchKernelGGL((k_forward<D, W, 2 * D + 1, ACT, PREC, true>), dim3(grid), dim3(64 * FwdWaves<W>::v), 0, st,
                         meta, centres, nets, L, h, outputs, Zst, Ast, ALst, lstride, noninline);
    else if (streams)
      hipLaunchKernelGGL((k_forward<D, W, 2 * D + 1, ACT, PREC, false>), dim3(grid), dim3(64 * FwdWaves<W>::v), 0, st,
                         meta, centres, nets, L, h, outputs, Zst, Ast, ALst, lstride, noninline);
    else
      hipLaunchKernelGGL((k_forward<D, W, 1, ACT, PREC, false>), dim3(grid), dim3(64 * FwdWaves<W>::v), 0, st, meta,
                         centres, nets, L, h, outputs, Zst, Ast, ALst, lstride, noninline);
    return hipGetLastError();
  }
  static hipError_t backward(hipStream_t st, int G, const Meta* meta, const float4* centres,
                             const Nets& nets, int L, int l, float h, const float* adj,
                             const float* Zst, const void* Ast, const float* ALst, float* dZ,
                             float* partial, int64_t Ptot, const NetLayout& lay, int64_t off1,
                             int64_t lstride) {
    hipLaunchKernelGGL((k_backward<D, W, ACT, PREC>), dim3(G), dim3(256), 0, st, meta, centres, nets,
                       L, l, h, adj, Zst, Ast, ALst, dZ, partial, Ptot, lay, off1, lstride);
    return hipGetLastError();
  }
};

template <int D>
hipError_t launch_sample(hipStream_t st, uint64_t seed, int64_t step, int64_t jh, float* pts,
                         int64_t n, float* bpts, int64_t nb) {
  int64_t tot = n + nb;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample<D>, dim3((tot + 255) / 256), dim3(256), 0, st, seed, step, jh, pts, n,
                     bpts, nb);
  return hipGetLastError();
}

#define NBM_FWD_BWD(D, W, ACT, PREC)                                                                \
  if (dim == D && width == W && act == ACT && prec == PREC) return &dispatch_impl<D, W, ACT, PREC>;

template <int D, int W, int ACT, int PREC>
hipError_t dispatch_impl(const MlpCall& c) {
  if (c.op == MlpCall::FORWARD)
    return Launch<D, W, ACT, PREC>::forward(c.stream, c.grid, c.meta, c.centres, *c.nets, c.L, c.h,
                                            c.outputs, c.Zst, c.Ast, c.ALst, c.lstride, c.store,
                                            c.streams, c.noninline);
  return Launch<D, W, ACT, PREC>::backward(c.stream, c.grid, c.meta, c.centres, *c.nets, c.L, c.l,
                                           c.h, c.adj, c.Zst, c.Ast, c.ALst, c.dZ, c.partial, c.Ptot,
                                           *c.lay, c.off1, c.lstride);
}

MlpFn find_mlp(int dim, int width, int act, int prec) {
  NBM_FWD_BWD(2, 16, 0, 0)
  NBM_FWD_BWD(2, 16, 1, 0)
  NBM_FWD_BWD(3, 16, 0, 0)
  NBM_FWD_BWD(3, 16, 1, 0)
  NBM_FWD_BWD(3, 64, 0, 0)
  NBM_FWD_BWD(3, 64, 1, 0)
  NBM_FWD_BWD(3, 64, 0, 1)
  NBM_FWD_BWD(3, 64, 1, 1)
  NBM_FWD_BWD(3, 128, 0, 0)
  NBM_FWD_BWD(3, 128, 1, 0)
  NBM_FWD_BWD(3, 128, 0, 1)
  NBM_FWD_BWD(3, 128, 1, 1)
  return nullptr;
}

// ---- non-MLP launchers ------------------------------------------------------
template <int D>
static void prep_impl(const PrepCall& c, int64_t nblk, int64_t nblkb) {
  hipStream_t st = c.stream;
  const int spm = c.shadows.count ? (c.shadows.W * c.shadows.W + 255) / 256 : 1;
  const int64_t nsh = (int64_t)c.shadows.count * spm;
  if (c.n + c.nb + nsh)
    hipLaunchKernelGGL(k_classify<D>, dim3(nblk + nblkb + nsh), dim3(256), 0, st, c.P, c.pts, c.n,
                       c.eval ? 1 : 0, c.tile_index, c.grid_n, c.cls, c.rank, c.blockcnt, (int)nblk,
                       c.bpts, c.nb, c.bcls, c.brank, c.blockcnt_b, (int)(nblk + nblkb), c.shadows,
                       c.prec, spm);
  // up to 2048 point blocks one work-group scans the block counts, 256 threads
  // when each count array fits one chunk of 256, else kScanThreads (one or two
  // chunks); larger
  // batches (evaluation tiles, the largest training batches) scan chunks of
  // kScanThreads counts in parallel, then the chunk totals
  const bool chunked = nblk + nblkb > 2048;
  const int64_t nci = (nblk + kScanThreads - 1) / kScanThreads, ncb = (nblkb + kScanThreads - 1) / kScanThreads;
  if (chunked) {
    hipLaunchKernelGGL(k_scan_chunks, dim3(nci + ncb), dim3(kScanThreads), 0, st, c.blockcnt, (int)nblk,
                       c.blockcnt_b, (int)nblkb, c.off, c.off_b, c.ctot, c.ctot_b, (int)nci);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(256), 0, st, c.ctot, (int)nci, c.ctot_b, (int)ncb, c.coff,
                       c.coff_b, c.meta, (int)c.n, (int)c.nb, c.cut_cap, D, c.P.lo, c.eval ? 1 : 0);
  } else {
    const int sthreads = nblk > 256 || nblkb > 256 ? kScanThreads : 256;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(sthreads), 0, st, c.blockcnt, (int)nblk, c.blockcnt_b,
                       (int)nblkb, c.off, c.off_b, c.meta, (int)c.n, (int)c.nb, c.cut_cap, D, c.P.lo,
                       c.eval ? 1 : 0);
  }
  if (c.n + c.nb)
    hipLaunchKernelGGL(k_scatter<D>, dim3(nblk + nblkb), dim3(256), 0, st, c.P, c.meta, c.pts, c.n,
                       c.cls, c.rank, c.off, c.tile_index, c.grid_n, c.centres, c.src, c.cutidx,
                       (int)nblk, c.bpts, c.nb, c.bcls, c.brank, c.off_b, c.fslot,
                       chunked ? c.coff : nullptr, chunked ? c.coff_b : nullptr);
}

hipError_t launch_prep(const PrepCall& c) {
  int64_t nblk = (c.n + 255) / 256, nblkb = (c.nb + 255) / 256;
  if (c.P.dim == 2) prep_impl<2>(c, nblk, nblkb);
  else prep_impl<3>(c, nblk, nblkb);
  return hipGetLastError();
}

hipError_t launch_residuals(const ResCall& c) {
  hipStream_t st = c.stream;
  int64_t nblk = (c.n + 255) / 256, nblkb = (c.nb + 255) / 256, nblkc = cut_blocks(c.cut_cap);
  double* lp = c.lossp;
  const int nblk_u = c.n ? (int)nblk : 0, nblk_c = c.n ? (int)nblkc : 0;
  const int64_t grid = (int64_t)nblk_u + nblk_c + (c.nb ? nblkb : 0);
  if (grid > 0) {
    if (c.P.dim == 2)
      hipLaunchKernelGGL(k_residuals<2>, dim3(grid), dim3(256), 0, st, c.P, c.meta, c.pts, c.n, c.cls, c.rank,
                         c.cutidx, c.bpts, c.nb, c.bcls, c.brank, c.outputs, c.adj, c.resid, lp, c.scale,
                         c.skip_inline, c.fpre, nblk_u, nblk_c);
    else
      hipLaunchKernelGGL(k_residuals<3>, dim3(grid), dim3(256), 0, st, c.P, c.meta, c.pts, c.n, c.cls, c.rank,
                         c.cutidx, c.bpts, c.nb, c.bcls, c.brank, c.outputs, c.adj, c.resid, lp, c.scale,
                         c.skip_inline, c.fpre, nblk_u, nblk_c);
  }
  if (c.loss) {
    int nparts = (int)(nblk + nblkc + nblkb) + c.extra_parts;
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(256), 0, st, c.lossp, nparts, c.meta, c.loss, c.lacc,
                       c.acc);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_loss(hipStream_t st, const double* lossp, int nparts, const Meta* meta,
                              double* loss) {
  hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(256), 0, st, lossp, nparts, meta, loss, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_forcing(hipStream_t st, const Problem& P, const float* pts, int64_t n, float* f,
                          const Meta* meta, const int* cls, const int* rank, float* fslot) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kForcingThreads - 1) / kForcingThreads)), block(kForcingThreads);
  if (P.dim == 2)
    hipLaunchKernelGGL(k_forcing<2>, grid, block, 0, st, P, pts, n, f, meta, cls, rank, fslot);
  else
    hipLaunchKernelGGL(k_forcing<3>, grid, block, 0, st, P, pts, n, f, meta, cls, rank, fslot);
  return hipGetLastError();
}

hipError_t launch_fill(hipStream_t st, float* p, int64_t n, float v) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, const float* partial, int G, int64_t P, float* grad,
                         double scale, const double* lossp, int nparts, const Meta* meta, double* loss,
                         double* gacc, double* lacc, int acc) {
  const int nblk = (int)((P + 63) / 64) + (loss ? 1 : 0);
  hipLaunchKernelGGL(k_reduce, dim3(nblk), dim3(1024), 0, st, partial, G, P, grad, scale, lossp, nparts,
                     meta, loss, gacc, lacc, acc);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t st, float* p, float* m, float* v, const float* g, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, m, v, g, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_sample_points(hipStream_t st, int dim, uint64_t seed, int64_t step, int64_t jh,
                                float* pts, int64_t n, float* bpts, int64_t nb) {
  return dim == 2 ? launch_sample<2>(st, seed, step, jh, pts, n, bpts, nb)
                  : launch_sample<3>(st, seed, step, jh, pts, n, bpts, nb);
}

hipError_t launch_counts(hipStream_t st, const Meta* meta, int* counts) {
  hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, meta, counts);
  return hipGetLastError();
}

hipError_t launch_eval_out(hipStream_t st, int64_t slots, const Meta* meta, const float* outputs,
                           const int* src, float* u_out) {
  hipLaunchKernelGGL(k_eval_out, dim3((slots + 255) / 256), dim3(256), 0, st, meta, outputs, src,
                     u_out);
  return hipGetLastError();
}

}  // namespace nbm
