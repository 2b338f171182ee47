// Evaluation of the trained surrogate, u(x) = u^{sigma(x)}(x): the base
// stream of each network's forward pass at the centres the preparation
// kernels compacted per network (queries, or coordinates generated from a
// grid tile index).
//
// Persistent work-groups of W/16 wavefronts; wavefront w owns neurons
// 16w..16w+15 of every layer and keeps its MFMA B operands of all hidden
// layers in registers for the whole launch (one load per network instead of
// one per tile).  Work-groups walk 64-centre tiles:
//   * layer 1 (K = d) on the VALU, activations to LDS rows [centre][neuron];
//   * hidden layers on MFMA, four 16-centre row blocks per wavefront, A rows
//     from LDS (double-buffered between layers), bias + activation in the
//     accumulator layout;
//   * output layer: w_out . a_L as one row sum per wavefront and centre, the
//     wavefronts' partials added in a fixed order, u written straight to the
//     query's position.
// The next tile's centres and query indices are fetched one tile ahead.
#include <hip/hip_runtime.h>

#include "nbm_device.hpp"
#include "nbm_internal.hpp"
#include "nbm_launch.hpp"

namespace nbm {

constexpr int kEvalTile = 64;   // centres per tile: four MFMA row blocks

template <int D, int W, int L, int ACT, int PREC>
__global__ __launch_bounds__(W * 4, PREC == 1 ? 2 : 1) void k_eval_mlp(const Meta* meta, const float4* centres,
                                                    const int* src, Nets nets, float* u_out) {
  typedef typename Op<PREC>::T T;
  constexpr int NW = W / 16;              // wavefronts = 16-neuron blocks
  constexpr int NT = W * 4;               // threads
  constexpr int RB = kEvalTile / 16;      // MFMA row blocks per tile
  constexpr int KC = W / 4;               // K chunk per lane group
  constexpr int LD = W + (PREC == 0 ? 4 : 8);
  constexpr int NB = PREC == 0 ? KC : KC / 8;   // B operand registers per layer
  static_assert(kEvalTile <= NT, "one thread per centre for the tile's bookkeeping");
  __shared__ __attribute__((aligned(16))) T buf[2][kEvalTile][LD];
  __shared__ float xs[kEvalTile][4];
  __shared__ int qs[kEvalTile];           // query index of each centre, -1 = padding
  __shared__ float part[NW][kEvalTile];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, g = lane >> 4;
  const int n = w * 16 + r16;             // neuron owned by this lane
  const int G = gridDim.x;

  for (int net = 0; net < 2; ++net) {
    const NetPtrs& np = nets.net[net];
    const int64_t s_lo = (int64_t)meta->tile0[net] * kTile;
    const int64_t s_hi = s_lo + meta->total[net];
    const int ntiles = (int)((meta->total[net] + kEvalTile - 1) / kEvalTile);
    if (ntiles == 0) continue;

    // this lane's B operands (row n of W_l, K chunk g) of every hidden layer
    struct BRows { float f[PREC == 0 ? L - 1 : 1][PREC == 0 ? NB : 1]; bf8 b[PREC == 1 ? L - 1 : 1][PREC == 1 ? NB : 1]; };
    BRows B;
#pragma unroll
    for (int l = 0; l < L - 1; ++l) {
      if constexpr (PREC == 0) {
        const float4* wp = (const float4*)((const float*)np.Wl[l] + (int64_t)n * W + g * KC);
#pragma unroll
        for (int q = 0; q < KC / 4; ++q) {
          const float4 v = wp[q];
          B.f[l][4 * q] = v.x; B.f[l][4 * q + 1] = v.y; B.f[l][4 * q + 2] = v.z; B.f[l][4 * q + 3] = v.w;
        }
      } else {
        const bf8* wp = (const bf8*)((const T*)np.Wl[l] + (int64_t)n * W + g * KC);
#pragma unroll
        for (int q = 0; q < NB; ++q) B.b[l][q] = wp[q];
      }
    }
    float bl[L - 1];
#pragma unroll
    for (int l = 0; l < L - 1; ++l) bl[l] = np.bl[l][n];
    float W1n[3] = {0.f, 0.f, 0.f};
    for (int a = 0; a < D; ++a) W1n[a] = np.W1[n * D + a];
    const float b1n = np.b1[n], won = np.wout[n], bout = np.bout[0];

    // next tile's centre and query index (thread c < kEvalTile holds centre c)
    float4 nx = make_float4(0.f, 0.f, 0.f, 0.f);
    int nq = -1;
    auto fetch = [&](int tt) {
      if (tt >= ntiles || tid >= kEvalTile) return;
      const int64_t s = s_lo + (int64_t)tt * kEvalTile + tid;
      const bool ok = s < s_hi;
      nx = ok ? centres[s] : make_float4(0.f, 0.f, 0.f, 0.f);
      nq = ok ? src[s] : -1;
    };
    fetch(blockIdx.x);

    for (int t = blockIdx.x; t < ntiles; t += G) {
      if (tid < kEvalTile) {
        xs[tid][0] = nx.x; xs[tid][1] = nx.y; xs[tid][2] = nx.z; xs[tid][3] = 0.f;
        qs[tid] = nq;
      }
      fetch(t + G);
      __syncthreads();

      // ---- layer 1 (VALU): centres 16 rb + 4 g + j of neuron n
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = 16 * rb + 4 * g + j;
          float z = b1n;
          for (int a = 0; a < D; ++a) z = fmaf(W1n[a], xs[c][a], z);
          buf[0][c][n] = from_f<T>(act_base<ACT>(z));
        }
      __syncthreads();

      // ---- hidden layers on MFMA; the last one feeds the output row sums
      float outp[RB][4];
      int cur = 0;
#pragma unroll
      for (int l = 0; l < L - 1; ++l) {
        f4 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if constexpr (PREC == 0) {
            const float4* ap = (const float4*)(&buf[cur][16 * rb + r16][g * KC]);
#pragma unroll
            for (int q = 0; q < KC / 4; ++q) {
              const float4 a4 = ap[q];
              acc[rb] = mfma4(a4.x, B.f[l][4 * q], acc[rb]);
              acc[rb] = mfma4(a4.y, B.f[l][4 * q + 1], acc[rb]);
              acc[rb] = mfma4(a4.z, B.f[l][4 * q + 2], acc[rb]);
              acc[rb] = mfma4(a4.w, B.f[l][4 * q + 3], acc[rb]);
            }
          } else {
            const bf8* ap = (const bf8*)(&buf[cur][16 * rb + r16][g * KC]);
#pragma unroll
            for (int q = 0; q < NB; ++q) acc[rb] = mfma32(ap[q], B.b[l][q], acc[rb]);
          }
        }
        const bool last = l == L - 2;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float a = act_base<ACT>(acc[rb][j] + bl[l]);
            if (last) outp[rb][j] = won * a;
            else buf[cur ^ 1][16 * rb + 4 * g + j][n] = from_f<T>(a);
          }
        if (!last) __syncthreads();
        cur ^= 1;
      }

      // ---- output layer: this wavefront's 16 neurons, then the wavefronts in order
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = row16_sum(outp[rb][j]);
          if (r16 == 0) part[w][16 * rb + 4 * g + j] = v;
        }
      __syncthreads();
      if (tid < kEvalTile && qs[tid] >= 0) {
        float u = part[0][tid];
        for (int v = 1; v < NW; ++v) u += part[v][tid];
        u_out[qs[tid]] = u + bout;
      }
      // The next tile rewrites xs and qs before its first barrier: every
      // wave's xs reads precede the barrier above, and qs[c] is read and
      // rewritten by thread c alone.  part and the row buffers are rewritten
      // only after that first barrier.
    }
    __syncthreads();
  }
}

// The work-groups loop over tiles, so the grid is what the device holds at
// once (work-groups per compute unit from the occupancy query, times the
// compute units), capped by the caller's bound on the tile count.
template <int D, int W, int L, int ACT, int PREC>
hipError_t eval_impl(const EvalCall& c) {
  static int resident = 0;   // per kernel instance; the library drives one device
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eval_mlp<D, W, L, ACT, PREC>, W * 4, 0);
    if (e != hipSuccess) return e;
    resident = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  }
  const int grid = c.max_grid < resident ? c.max_grid : resident;
  hipLaunchKernelGGL((k_eval_mlp<D, W, L, ACT, PREC>), dim3(grid), dim3(W * 4), 0, c.stream, c.meta,
                     c.centres, c.src, *c.nets, c.u_out);
  return hipGetLastError();
}

#define NBM_EVAL(D, W, L, ACT, PREC) \
  if (dim == D && width == W && depth == L && act == ACT && prec == PREC) return &eval_impl<D, W, L, ACT, PREC>;

EvalFn find_eval(int dim, int width, int depth, int act, int prec) {
  NBM_EVAL(3, 64, 3, 0, 0)
  NBM_EVAL(3, 64, 3, 1, 0)
  NBM_EVAL(3, 64, 3, 0, 1)
  NBM_EVAL(3, 64, 3, 1, 1)
  NBM_EVAL(3, 128, 4, 0, 0)
  NBM_EVAL(3, 128, 4, 1, 0)
  NBM_EVAL(3, 128, 4, 0, 1)
  NBM_EVAL(3, 128, 4, 1, 1)
  return nullptr;
}

}  // namespace nbm
