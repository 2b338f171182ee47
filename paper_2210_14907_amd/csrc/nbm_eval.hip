// Evaluation of the trained surrogate, u(x) = u^{sigma(x)}(x): the base
// stream of each network's forward pass at the centres the preparation
// kernels compacted per network (queries, or coordinates generated from a
// grid tile index).
//
// Persistent work-groups; each wavefront owns two 16-neuron blocks of every
// layer (one for FP32 operands of 128-wide nets) and keeps its rows of all
// hidden weight matrices in registers for the whole launch (one load per network instead
// of one per tile).  Each product is formed transposed, Z^T = W A^T: the
// weights are the MFMA's A operand and the activation rows [centre][neuron]
// in LDS its B operand, so a lane's accumulators hold four consecutive
// neurons of one centre.  Work-groups walk 64-centre tiles:
//   * layer 1 (K = d) on the VALU;
//   * hidden layers on MFMA over four 16-centre blocks, activations written
//     back as one 4-neuron vector per lane and block (double-buffered rows);
//   * output layer: w_out . a_L over the lane's four neurons, then across
//     the lane groups and, in a fixed order, the wavefronts; u is written
//     straight to the query's position.
// The next tile's centres and query indices are fetched one tile ahead.
#include <hip/hip_runtime.h>

#include "nbm_device.hpp"
#include "nbm_internal.hpp"
#include "nbm_launch.hpp"

namespace nbm {

constexpr int kEvalTile = 64;   // centres per tile: four MFMA row blocks

// 16-neuron blocks per wavefront: two, so that each activation operand read
// from LDS feeds two products (half the LDS traffic of one block per
// wavefront), unless the FP32 operands of a 128-wide net would not fit
template <int W, int PREC> struct EvalShape {
  static constexpr int NBW = (PREC == 0 && W >= 128) ? 1 : 2;
  static constexpr int NW = W / (16 * NBW);   // wavefronts
  static constexpr int NT = NW * 64;          // threads
};

template <int D, int W, int L, int ACT, int PREC>
__global__ __launch_bounds__((EvalShape<W, PREC>::NT), 2) void k_eval_mlp(const Meta* meta, const float4* centres,
                                                                       const int* src, Nets nets, float* u_out) {
  typedef typename Op<PREC>::T T;
  constexpr int NBW = EvalShape<W, PREC>::NBW;
  constexpr int NW = EvalShape<W, PREC>::NW;
  constexpr int NT = EvalShape<W, PREC>::NT;
  constexpr int RB = kEvalTile / 16;      // MFMA row blocks per tile
  constexpr int KC = W / 4;               // K chunk per lane group
  constexpr int NB = PREC == 0 ? KC : KC / 8;   // operand registers per layer and block
  static_assert(kEvalTile <= NT, "one thread per centre for the tile's bookkeeping");
  // Activation tiles, the B operand of every product.  BF16: per 16-centre
  // row block, the 16-byte chunk k (neurons 8k .. 8k+7) of its 16 centres
  // side by side, and lane group g takes chunk 4q + g at step q, so one
  // operand read covers 1 KB in lane order (padded centre rows cost extra
  // LDS bank-conflict cycles on every read).  FP32: centre rows padded to
  // W + 4, lane group g taking neurons g W/4 + 4q .. + 3.
  constexpr int kBuf = PREC == 1 ? kEvalTile * W : kEvalTile * (W + 4);
  __shared__ __attribute__((aligned(16))) T buf[2][kBuf];
  // position of (centre c, neuron m), and of the operand of lane (r, gg) of
  // row block rb at step q
  auto bpos = [](int c, int m) {
    return PREC == 1 ? (((c >> 4) * (W / 8) + (m >> 3)) * 16 + (c & 15)) * 8 + (m & 7) : c * (W + 4) + m;
  };
  auto opos = [](int rb, int r, int gg, int q) {
    return PREC == 1 ? ((rb * (W / 8) + 4 * q + gg) * 16 + r) * 8 : (16 * rb + r) * (W + 4) + gg * KC + 4 * q;
  };
  __shared__ float xs[kEvalTile][4];
  __shared__ int qs[kEvalTile];           // query index of each centre, -1 = padding
  __shared__ float part[NW][kEvalTile];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, g = lane >> 4;
  const int G = gridDim.x;
  // neuron block k of this wavefront: neurons 16 (NBW w + k) + 0..15
  auto blk = [&](int k) { return NBW * w + k; };
  // sin networks: weights and biases of layers 1..L times 1/(2 pi), so every
  // pre-activation is in revolutions, the unit of the hardware sine
  constexpr float ks = ACT == 1 ? 0.15915494309189535f : 1.0f;
  auto act = [](float z) {
    if constexpr (ACT == 1) return __builtin_amdgcn_sinf(z);
    else return tanh_base(z).t;
  };

  for (int net = 0; net < 2; ++net) {
    const NetPtrs& np = nets.net[net];
    const int64_t s_lo = (int64_t)meta->tile0[net] * kTile;
    const int64_t s_hi = s_lo + meta->total[net];
    const int ntiles = (int)((meta->total[net] + kEvalTile - 1) / kEvalTile);
    if (ntiles == 0) continue;

    // this lane's A operands (row 16 blk(k) + r16 of W_l, K chunk g) of every
    // hidden layer and block, from the FP32 master weights times ks, rounded
    // once to the operand type
    struct WRows { float f[PREC == 0 ? L - 1 : 1][NBW][PREC == 0 ? NB : 1]; bf8 b[PREC == 1 ? L - 1 : 1][NBW][PREC == 1 ? NB : 1]; };
    WRows A;
#pragma unroll
    for (int l = 0; l < L - 1; ++l)
#pragma unroll
      for (int k = 0; k < NBW; ++k) {
        // FP32: K values g W/4 + 4q + i; BF16: operand q takes the chunk
        // 4q + g of the row (the activation tiles' order)
        const float* wrow = np.Wf[l] + (int64_t)(16 * blk(k) + r16) * W;
#pragma unroll
        for (int q = 0; q < KC / 4; ++q) {
          const int e0 = PREC == 0 ? g * KC + 4 * q : 8 * (4 * (q / 2) + g) + 4 * (q & 1);
          const float4 v = *(const float4*)(wrow + e0);
          const float e[4] = {ks * v.x, ks * v.y, ks * v.z, ks * v.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if constexpr (PREC == 0) A.f[l][k][4 * q + i] = e[i];
            else A.b[l][k][q / 2][4 * (q & 1) + i] = (__bf16)e[i];
          }
        }
      }
    // the output neurons of this lane's accumulators: 16 blk(k) + 4 g + j
    float bl[L - 1][NBW][4], W1n[NBW][4][3], b1n[NBW][4], won[NBW][4];
#pragma unroll
    for (int k = 0; k < NBW; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int nn = 16 * blk(k) + 4 * g + j;
#pragma unroll
        for (int l = 0; l < L - 1; ++l) bl[l][k][j] = ks * np.bl[l][nn];
        for (int a = 0; a < 3; ++a) W1n[k][j][a] = a < D ? ks * np.W1[nn * D + a] : 0.f;
        b1n[k][j] = ks * np.b1[nn];
        won[k][j] = np.wout[nn];
      }
    const float bout = np.bout[0];

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

      // stores of a lane's four consecutive neurons of block k at centre c
      auto put4 = [&](int b, int c, int k, const float* v) {
        const int n0 = 16 * blk(k) + 4 * g;
        if constexpr (PREC == 0) *(float4*)(&buf[b][bpos(c, n0)]) = make_float4(v[0], v[1], v[2], v[3]);
        else *(bf4*)(&buf[b][bpos(c, n0)]) = bf4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
      };

      // ---- layer 1 (VALU): centre 16 rb + r16, neurons 16 blk(k) + 4 g + j
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int c = 16 * rb + r16;
#pragma unroll
        for (int k = 0; k < NBW; ++k) {
          float v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float z = b1n[k][j];
            for (int a = 0; a < D; ++a) z = fmaf(W1n[k][j][a], xs[c][a], z);
            v[j] = act(z);
          }
          put4(0, c, k, v);
        }
      }
      __syncthreads();

      // ---- hidden layers on MFMA; the last one feeds the output sums
      float outp[RB];
      int cur = 0;
#pragma unroll
      for (int l = 0; l < L - 1; ++l) {
        f4 acc[NBW][RB];
#pragma unroll
        for (int k = 0; k < NBW; ++k)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) acc[k][rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if constexpr (PREC == 0) {
            const float4* bp = (const float4*)(&buf[cur][opos(rb, r16, g, 0)]);
#pragma unroll
            for (int q = 0; q < KC / 4; ++q) {
              const float4 b4 = bp[q];
#pragma unroll
              for (int k = 0; k < NBW; ++k) {
                acc[k][rb] = mfma4(A.f[l][k][4 * q], b4.x, acc[k][rb]);
                acc[k][rb] = mfma4(A.f[l][k][4 * q + 1], b4.y, acc[k][rb]);
                acc[k][rb] = mfma4(A.f[l][k][4 * q + 2], b4.z, acc[k][rb]);
                acc[k][rb] = mfma4(A.f[l][k][4 * q + 3], b4.w, acc[k][rb]);
              }
            }
          } else {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
              const bf8 b8 = *(const bf8*)(&buf[cur][opos(rb, r16, g, q)]);
#pragma unroll
              for (int k = 0; k < NBW; ++k) acc[k][rb] = mfma32(A.b[l][k][q], b8, acc[k][rb]);
            }
          }
        }
        const bool last = l == L - 2;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          float o = 0.f;
#pragma unroll
          for (int k = 0; k < NBW; ++k) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = act(acc[k][rb][j] + bl[l][k][j]);
            if (last) {
#pragma unroll
              for (int j = 0; j < 4; ++j) o = fmaf(won[k][j], v[j], o);
            } else {
              put4(cur ^ 1, 16 * rb + r16, k, v);
            }
          }
          if (last) outp[rb] = o;
        }
        if (!last) __syncthreads();
        cur ^= 1;
      }

      // ---- output layer: the four lane groups (same centre), then the
      // wavefronts in order
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        float v = outp[rb];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (g == 0) part[w][16 * rb + r16] = v;
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
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eval_mlp<D, W, L, ACT, PREC>,
                                                       EvalShape<W, PREC>::NT, 0);
    if (e != hipSuccess) return e;
    resident = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  }
  const int grid = c.max_grid < resident ? c.max_grid : resident;
  hipLaunchKernelGGL((k_eval_mlp<D, W, L, ACT, PREC>), dim3(grid), dim3(EvalShape<W, PREC>::NT), 0, c.stream, c.meta,
                     c.centres, c.src, *c.nets, c.u_out);
  return hipGetLastError();
}

// Grid fallback of the evaluation: at every point of tile `tile` (m
// consecutive points of the grid_n^D lattice x_a = -1 + 2 i_a / grid_n, axis 0
// fastest), the multilinear interpolation of a nodal solution U given on the
// (judge_n + 1)^D nodes y_a = -1 + 2 j_a / judge_n (axis 0 fastest).  FP64
// weights and sums, FP32 output.  One thread per point; consecutive threads
// read neighbouring nodes, so a wavefront's loads of U stay within a few
// cache lines of each row.
template <int D>
__global__ __launch_bounds__(256) void k_grid_interp(const double* __restrict__ U, int judge_n, int64_t first,
                                                     int64_t m, int grid_n, float* __restrict__ u_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int64_t q = first + i;
  const double scale = (double)judge_n / (double)grid_n;   // judge intervals per lattice step
  int j0[D];
  double fr[D];
  for (int a = 0; a < D; ++a) {
    const int64_t ia = q % grid_n;
    q /= grid_n;
    const double t = (double)ia * scale;                 // position in judge cells
    int j = (int)t;
    if (j > judge_n - 1) j = judge_n - 1;
    j0[a] = j;
    fr[a] = t - (double)j;
  }
  const int64_t s1 = judge_n + 1, s2 = s1 * s1;
  double acc = 0.0;
  for (int c = 0; c < (1 << D); ++c) {
    double w = 1.0;
    int64_t flat = 0;
    for (int a = 0; a < D; ++a) {
      const int bit = (c >> a) & 1;
      w *= bit ? fr[a] : 1.0 - fr[a];
      flat += (int64_t)(j0[a] + bit) * (a == 0 ? 1 : (a == 1 ? s1 : s2));
    }
    acc += w * U[flat];
  }
  u_out[i] = (float)acc;
}

hipError_t launch_grid_interp(hipStream_t st, int dim, const double* U, int judge_n, int64_t tile_index,
                              int64_t m, int grid_n, float* u_out) {
  const dim3 grid((unsigned)((m + 255) / 256)), block(256);
  const int64_t first = tile_index * m;
  if (dim == 2)
    hipLaunchKernelGGL(k_grid_interp<2>, grid, block, 0, st, U, judge_n, first, m, grid_n, u_out);
  else
    hipLaunchKernelGGL(k_grid_interp<3>, grid, block, 0, st, U, judge_n, first, m, grid_n, u_out);
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
