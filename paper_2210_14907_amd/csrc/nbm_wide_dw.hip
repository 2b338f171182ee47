// Pass 2 of the 128-wide training step: the weight gradients dW_l of the
// hidden layers from the operand rows A_{l-1} and dZ_l that the forward/
// backward pass (nbm_wide.hip) stored in the tile layout
// [tile][stream][neuron][16 centres].  dW_l = sum over (tile, stream, centre)
// of dZ_l^T A_{l-1}, read straight from that layout as MFMA operands (the K
// index runs over stream pairs x 4 centres per lane group), split over
// persistent work-groups that each write one partial row; the FP64
// reduction follows.  Built in a translation unit of its own: the compiler's
// ILP scheduling strategy removes this kernel's register spills (2-3 %
// faster), while the forward/backward kernel is slower under it.
#include <hip/hip_runtime.h>

#include "nbm_device.hpp"
#include "nbm_internal.hpp"
#include "nbm_launch.hpp"

namespace nbm {

// dW_l partials.  A work-group of 8 wavefronts: waves w and w+4 (one SIMD)
// form two halves that take alternate tiles (twice the loads in flight);
// within a half, wave w owns out-blocks {w, w+4, ...} and all in-blocks.  The
// halves' accumulators are added in a fixed order through LDS at the end.
// BF16: each half stages the A block of its tile in LDS once (double-
// buffered, the next tile's block in flight during the current MFMAs)
// instead of every wave reading all of it from L2.  For the first hidden
// layer (A1) the block is not read at all: the first layer's activation
// streams of the tile's centres are recomputed from the centres and W_1, b_1
// (the same arithmetic as the forward pass, rounded to BF16 the same way),
// which spares the forward pass their stores and this pass their reads.
template <int D, int W, int PREC, int ACT, bool A1>
__global__ __launch_bounds__(512) void k_wide_dw(const Meta* meta, const void* A_, const void* dZ_,
                                                 float* partial, int64_t Ptot, int64_t woff,
                                                 int64_t net_off1, const float4* centres, Nets nets,
                                                 float h) {
  static_assert(!A1 || PREC == 1, "the first layer's operand rows are rebuilt on the BF16 path");
  typedef typename Op<PREC>::T T;
  constexpr int S = 2 * D + 1;
  constexpr int NOB = W / 16;
  constexpr int OBW = NOB / 4;
  constexpr int TA = S * W * kTile;          // elements of one tile's A block
  constexpr int NQ = TA * 2 / 16 / 256;      // 16-byte pieces per lane of a half (BF16)
  static_assert(PREC == 0 || TA * 2 % (16 * 256) == 0, "A block splits into 16-byte pieces");
  const T* A = (const T*)A_;
  const T* dZ = (const T*)dZ_;
  const int tid = threadIdx.x, lane = tid & 63, w = (tid >> 6) & 3, half = tid >> 8, hl = tid & 255;
  const int r16 = lane & 15, g = lane >> 4;
  const int G = gridDim.x;
  // staging [half][buffer][TA] (BF16); after the tile loop the same bytes
  // hold the second half's accumulators
  constexpr int kStageBytes = PREC == 1 ? 2 * 2 * TA * 2 : 0;
  constexpr int kXchBytes = OBW * NOB * 256 * 16;
  __shared__ __attribute__((aligned(16))) char lds[kStageBytes > kXchBytes ? kStageBytes : kXchBytes];
  T* stage = reinterpret_cast<T*>(lds);
  // Staged A block: a row (one stream and input neuron, 16 centres, 32 bytes)
  // holds two 16-byte halves, swapped in rows whose index has bit 3 set.  A
  // wavefront's operand read takes 8 bytes from each of 16 consecutive rows
  // (two lane groups per half-wavefront); without the swap rows r and r + 8
  // fall on the same banks.
  auto stage_slot = [](int u) { const int row = u >> 1; return (row << 1) | ((u & 1) ^ ((row >> 3) & 1)); };
  f4 (*xch)[NOB][256] = reinterpret_cast<f4 (*)[NOB][256]>(lds);
  for (int net = 0; net < 2; ++net) {
    const int t_lo = net == 0 ? 0 : meta->tiles[0];
    const int t_hi = net == 0 ? meta->tiles[0] : meta->tiles[0] + meta->tiles[1];
    f4 acc[OBW][NOB];
    for (int i = 0; i < OBW; ++i)
      for (int k = 0; k < NOB; ++k) acc[i][k] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == 0) {
      for (int t = t_lo + blockIdx.x + half * G; t < t_hi; t += 2 * G) {
        auto tofs = [&](int s, int nn) -> int64_t { return (((int64_t)t * S + s) * W + nn) * kTile + 4 * g; };
        float dzv[OBW][S][4];
        for (int i = 0; i < OBW; ++i)
          for (int s = 0; s < S; ++s) {
            // (plain loads: streaming ones measured slower on this FP32 path)
            const f4 v = *(const f4*)(dZ + tofs(s, (w + 4 * i) * 16 + r16));
            dzv[i][s][0] = v.x; dzv[i][s][1] = v.y; dzv[i][s][2] = v.z; dzv[i][s][3] = v.w;
          }
        for (int ib = 0; ib < NOB; ++ib)
          for (int s = 0; s < S; ++s) {
            const f4 a = *(const f4*)(A + tofs(s, ib * 16 + r16));
            for (int i = 0; i < OBW; ++i) {
              acc[i][ib] = mfma4(dzv[i][s][0], a.x, acc[i][ib]);
              acc[i][ib] = mfma4(dzv[i][s][1], a.y, acc[i][ib]);
              acc[i][ib] = mfma4(dzv[i][s][2], a.z, acc[i][ib]);
              acc[i][ib] = mfma4(dzv[i][s][3], a.w, acc[i][ib]);
            }
          }
      }
    } else {
      // iterations: half 0 has at least as many tiles as half 1; both halves
      // run the same count so that their barriers pair up
      const int span = t_hi - t_lo - (int)blockIdx.x;
      const int niter = span > 0 ? (span + 2 * G - 1) / (2 * G) : 0;
      auto tile_of = [&](int k) { return t_lo + (int)blockIdx.x + half * G + 2 * G * k; };
      // the next tile's A block travels through registers; a half past its
      // last tile re-reads the net's last tile (in bounds, never used)
      u4 pre[A1 ? 1 : NQ];
      // A1: this thread rebuilds neuron an at centres ac0 .. ac0+7 of a tile
      const int an = hl >> 1, ac0 = (hl & 1) * 8;
      float aW1[3] = {0.f, 0.f, 0.f}, ab1 = 0.f;
      L1Axes aax{};
      if constexpr (A1) {
        const NetPtrs& np = nets.net[net];
        float p1[3] = {0.f, 0.f, 0.f};
        for (int a = 0; a < D; ++a) { aW1[a] = np.W1[an * D + a]; p1[a] = h * aW1[a]; }
        ab1 = np.b1[an];
        aax = l1_axes<ACT, D>(p1);
      }
      const int64_t slot_end = (int64_t)meta->tile0[net] * kTile + meta->total[net];
      auto build_A = [&](int t, T* dst) {
        if (t >= t_hi) return;
        const int64_t slot0 = (int64_t)t * kTile + ac0;
        bf8 o[S];
        for (int c = 0; c < 8; ++c) {
          float4 cc = slot0 + c < slot_end ? centres[slot0 + c] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float xc[3] = {cc.x, cc.y, cc.z};
          float z = ab1;
          for (int a = 0; a < D; ++a) z += aW1[a] * xc[a];
          float av, Dv[3], Ev[3];
          act_fwd_l1<ACT, D>(z, aax, av, Dv, Ev);
          o[0][c] = (__bf16)av;
          for (int a = 0; a < D; ++a) { o[1 + a][c] = (__bf16)Dv[a]; o[1 + D + a][c] = (__bf16)Ev[a]; }
        }
        for (int s = 0; s < S; ++s) {
          const int row = s * W + an;
          *(bf8*)(dst + row * kTile + (((ac0 >> 3) ^ ((row >> 3) & 1)) << 3)) = o[s];
        }
      };
      auto src_of = [&](int k) {
        const int t = tile_of(k) < t_hi ? tile_of(k) : t_hi - 1;
        return (const u4*)(A + (int64_t)t * TA);
      };
      // this lane's dZ rows of a tile (out-blocks w + 4i, every stream), also
      // one tile ahead; the offset within a tile block is a 32-bit lane value
      bf4 dzr[OBW][S];
      auto load_dz = [&](int k) {
        const int t = tile_of(k) < t_hi ? tile_of(k) : t_hi - 1;
        const char* tb = (const char*)(dZ + (int64_t)t * TA);
        for (int i = 0; i < OBW; ++i)
          for (int s = 0; s < S; ++s)
            dzr[i][s] = ld_stream((const bf4*)(tb + (uint32_t)((((s * W + (w + 4 * i) * 16 + r16) * kTile) + 4 * g) * 2)));
      };
      if (niter > 0) {
        if constexpr (A1) {
          build_A(tile_of(0), stage + (half * 2) * TA);
        } else {
          const u4* s4 = src_of(0);
#pragma unroll
          for (int q = 0; q < NQ; ++q) pre[q] = ld_stream(&s4[q * 256 + hl]);
          u4* d4 = (u4*)(stage + (half * 2) * TA);
#pragma unroll
          for (int q = 0; q < NQ; ++q) d4[stage_slot(q * 256 + hl)] = pre[q];
        }
        load_dz(0);
      }
      __syncthreads();
      const bf4 zero4 = bf4{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
      for (int k = 0; k < niter; ++k) {
        const int t = tile_of(k);
        bf8 dzv[OBW][(S + 1) / 2];
        for (int i = 0; i < OBW; ++i)
          for (int s = 0; s < S; s += 2) {
            const bf4 v0 = dzr[i][s];
            const bf4 v1 = s + 1 < S ? dzr[i][s + 1] : zero4;
            for (int j = 0; j < 4; ++j) { dzv[i][s / 2][j] = v0[j]; dzv[i][s / 2][4 + j] = v1[j]; }
          }
        {
          if constexpr (!A1) {
            const u4* s4 = src_of(k + 1);
#pragma unroll
            for (int q = 0; q < NQ; ++q) pre[q] = ld_stream(&s4[q * 256 + hl]);
          }
          load_dz(k + 1);
        }
        if (t < t_hi) {
          const T* As = stage + (half * 2 + (k & 1)) * TA;
          // centres 4g..4g+3 of a row: half (g >> 1) of it, swapped in rows with bit 3 set
          const int cofs = ((((g >> 1) ^ (r16 >> 3)) << 3) | ((g & 1) << 2));
          for (int ib = 0; ib < NOB; ++ib)
            for (int s = 0; s < S; s += 2) {
              bf4 v0 = *(const bf4*)(As + (s * W + ib * 16 + r16) * kTile + cofs);
              bf4 v1 = s + 1 < S ? *(const bf4*)(As + ((s + 1) * W + ib * 16 + r16) * kTile + cofs) : zero4;
              bf8 a;
              for (int j = 0; j < 4; ++j) { a[j] = v0[j]; a[4 + j] = v1[j]; }
              for (int i = 0; i < OBW; ++i) acc[i][ib] = mfma32(dzv[i][s / 2], a, acc[i][ib]);
            }
        }
        // the other buffer was last read in iteration k-1, before its barrier
        if constexpr (A1) {
          build_A(tile_of(k + 1), stage + (half * 2 + ((k + 1) & 1)) * TA);
        } else {
          u4* d4 = (u4*)(stage + (half * 2 + ((k + 1) & 1)) * TA);
#pragma unroll
          for (int q = 0; q < NQ; ++q) d4[stage_slot(q * 256 + hl)] = pre[q];
        }
        __syncthreads();
      }
    }
    // first half + second half, in that order
    if (half == 1)
      for (int i = 0; i < OBW; ++i)
        for (int ib = 0; ib < NOB; ++ib) xch[i][ib][hl] = acc[i][ib];
    __syncthreads();
    if (half == 0) {
      float* prow = partial + (int64_t)blockIdx.x * Ptot + (net == 0 ? 0 : net_off1) + woff;
      for (int i = 0; i < OBW; ++i)
        for (int ib = 0; ib < NOB; ++ib) {
          const f4 o = xch[i][ib][hl];
          for (int r = 0; r < 4; ++r) {
            int row = (w + 4 * i) * 16 + 4 * g + r, col = ib * 16 + r16;
            st_stream(&prow[(int64_t)row * W + col], acc[i][ib][r] + o[r]);
          }
        }
    }
    __syncthreads();
  }
}

// launches k_wide_dw for hidden layer l (2 .. L) of a wide_impl call
template <int D, int W, int PREC, int ACT>
hipError_t launch_wide_dw(const WideCall& c, int l) {
  const char* Al = (const char*)c.A + (int64_t)(l - 2) * c.lstride * Op<PREC>::bytes;
  const char* dZl = (const char*)c.dZ + (int64_t)(l - 2) * c.lstride * Op<PREC>::bytes;
  if (PREC == 1 && l == 2)   // BF16: the first layer's rows are rebuilt from the centres
    hipLaunchKernelGGL((k_wide_dw<D, W, PREC, ACT, PREC == 1>), dim3(c.grid), dim3(512), 0, c.stream,
                       c.meta, Al, dZl, c.partial, c.Ptot, c.lay->Wl[l - 2], c.off1, c.centres, *c.nets, c.h);
  else
    hipLaunchKernelGGL((k_wide_dw<D, W, PREC, ACT, false>), dim3(c.grid), dim3(512), 0, c.stream,
                       c.meta, Al, dZl, c.partial, c.Ptot, c.lay->Wl[l - 2], c.off1, c.centres, *c.nets, c.h);
  return hipGetLastError();
}

template hipError_t launch_wide_dw<3, 128, 1, 1>(const WideCall&, int);
template hipError_t launch_wide_dw<3, 128, 0, 1>(const WideCall&, int);
template hipError_t launch_wide_dw<3, 128, 1, 0>(const WideCall&, int);
template hipError_t launch_wide_dw<3, 128, 0, 0>(const WideCall&, int);

}  // namespace nbm
