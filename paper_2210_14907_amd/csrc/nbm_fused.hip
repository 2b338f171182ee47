// Fused forward + residual + backward over difference streams for W = 64
// networks: one persistent work-group walks 16-centre tiles, keeps every
// activation of the tile on chip (pre-activations in registers, GEMM operands
// in LDS in the two layouts the forward and dW contractions need) and
// accumulates dW in MFMA accumulators; nothing per layer touches HBM.
//
// Tile classes: an "inline" tile holds 16 uncut (class A) centres, whose
// residual -sum_i eu_i/h^2 - f/mu and adjoints are formed inside the kernel.
// Every other tile (cut cells, low-mu neighbour centres, boundary points,
// the ragged end of the uncut list) reads its output adjoints from the
// workspace, written beforehand by the residual kernels after a
// forward-only pass over those tiles.
#include <hip/hip_runtime.h>

#include "nbm_device.hpp"
#include "nbm_internal.hpp"
#include "nbm_launch.hpp"

namespace nbm {

__device__ inline int fused_tile_net(const Meta* m, int t) {
  if (t < m->tiles[0]) return 0;
  if (t < m->tiles[0] + m->tiles[1]) return 1;
  return -1;
}

template <int D, int W, int L, int ACT, int PREC>
__global__ __launch_bounds__(256) void k_fused(const Meta* meta, const float4* centres, const int* src,
                                               Nets nets, Problem P, float h, const float* adj,
                                               float* resid, float* partial, int64_t Ptot,
                                               NetLayout lay, int64_t net_off1, double* lossp,
                                               double scale, const float* fpre) {
  typedef typename Op<PREC>::T T;
  constexpr int S = 2 * D + 1;
  constexpr int LD = W + (PREC == 0 ? 4 : 8);
  constexpr int NOB = W / 16;       // 16-neuron blocks; wave w owns block w
  constexpr int KC = W / 4;         // K chunk per lane group
  static_assert(NOB == 4, "one 16-neuron block per wave");
  __shared__ __attribute__((aligned(16))) T bufR[2][S][kTile][LD];      // row layout [c][n]
  constexpr int CP = kTile + (PREC == 0 ? 4 : 8);   // padded column stride
  __shared__ __attribute__((aligned(16))) T colA[L - 1][S][W][CP];      // column layout [n][c]
  __shared__ __attribute__((aligned(16))) float colL[S][W][kTile];   // last-layer activations (FP32)
  __shared__ float adjs[kTile][8];
  // output-layer partial sums live in the row buffers, free between the last
  // forward layer and the first backward write
  float (*part)[kTile][8] = reinterpret_cast<float (*)[kTile][8]>(&bufR[0][0][0][0]);
  static_assert(sizeof(bufR) >= 4 * kTile * 8 * sizeof(float), "partials fit the row buffers");
  __shared__ float xs[kTile][4];
  __shared__ double lsum[kTile];
  __shared__ int tflag;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, g = lane >> 4;
  const int n = w * 16 + r16;   // neuron owned by this lane, centres 4g..4g+3
  const int G = gridDim.x;
  const int ntiles = meta->tiles[0] + meta->tiles[1];
  const float hh = h * h;
  if (tid < kTile) lsum[tid] = 0.0;

  for (int net = 0; net < 2; ++net) {
    const NetPtrs& np = nets.net[net];
    f4 accW[L - 1][NOB];
    float accb[L], accW1[3] = {0.f, 0.f, 0.f}, accwo = 0.f, accbo = 0.f;
    for (int l = 0; l < L - 1; ++l)
      for (int k = 0; k < NOB; ++k) accW[l][k] = f4{0.f, 0.f, 0.f, 0.f};
    for (int l = 0; l < L; ++l) accb[l] = 0.f;
    float W1n[3], p1[3], e0[3] = {0.f, 0.f, 0.f};
    for (int a = 0; a < D; ++a) { W1n[a] = np.W1[n * D + a]; p1[a] = h * W1n[a]; }
    const float b1n = np.b1[n], won = np.wout[n];
    const int64_t a_end = (int64_t)meta->base[net][KIND_A] + meta->cnt[net][KIND_A];

    for (int t = blockIdx.x; t < ntiles; t += G) {
      if (fused_tile_net(meta, t) != net) continue;
      const int64_t slot0 = (int64_t)t * kTile;
      const int64_t slot_end = (int64_t)meta->tile0[net] * kTile + meta->total[net];
      if (tid < kTile) {
        float4 cc = centres[slot0 + tid];
        if (slot0 + tid >= slot_end) cc = make_float4(0.f, 0.f, 0.f, 0.f);
        xs[tid][0] = cc.x; xs[tid][1] = cc.y; xs[tid][2] = cc.z; xs[tid][3] = 0.f;
      }
      if (tid == 0) tflag = (slot0 + kTile <= a_end) ? 1 : 0;
      __syncthreads();
      const bool inl = tflag != 0;

      // ---------------- forward, layer 1 (VALU, accumulator mapping)
      float z1[4];
      for (int j = 0; j < 4; ++j) {
        int c = 4 * g + j;
        float z = b1n;
        for (int a = 0; a < D; ++a) z += W1n[a] * xs[c][a];
        z1[j] = z;
        float av, Dv[3], Ev[3];
        act_fwd<ACT, D>(z, p1, e0, av, Dv, Ev);
        float vals[7];
        vals[0] = av;
        for (int a = 0; a < D; ++a) { vals[1 + a] = Dv[a]; vals[1 + D + a] = Ev[a]; }
        for (int s = 0; s < S; ++s) {
          T v = from_f<T>(vals[s]);
          bufR[0][s][c][n] = v;
          colA[0][s][n][c] = v;
        }
      }
      __syncthreads();

      // ---------------- forward, hidden layers on MFMA
      float Z[L - 1][S][4];   // pre-activations of layers 2..L for (centres 4g+j, neuron n)
      int cur = 0;
#pragma unroll
      for (int l = 2; l <= L; ++l) {
        f4 acc[S];
        for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == 0) {
          float bk[KC];
          const float4* wp = (const float4*)((const float*)np.Wl[l - 2] + (int64_t)n * W + g * KC);
          for (int q = 0; q < KC / 4; ++q) {
            float4 v4 = wp[q];
            bk[4 * q] = v4.x; bk[4 * q + 1] = v4.y; bk[4 * q + 2] = v4.z; bk[4 * q + 3] = v4.w;
          }
          for (int s = 0; s < S; ++s) {
            const float4* ap = (const float4*)(&bufR[cur][s][r16][g * KC]);
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
          const bf8* wp = (const bf8*)((const T*)np.Wl[l - 2] + (int64_t)n * W + g * KC);
          for (int q = 0; q < KC / 8; ++q) bk[q] = wp[q];
          for (int s = 0; s < S; ++s) {
            const bf8* ap = (const bf8*)(&bufR[cur][s][r16][g * KC]);
            for (int q = 0; q < KC / 8; ++q) acc[s] = mfma32(ap[q], bk[q], acc[s]);
          }
        }
        const float bias = np.bl[l - 2][n];
        const bool last = (l == L);
        for (int j = 0; j < 4; ++j) {
          int c = 4 * g + j;
          float z = acc[0][j] + bias;
          float pp[3], ee[3], av, Dv[3], Ev[3];
          for (int a = 0; a < D; ++a) { pp[a] = acc[1 + a][j]; ee[a] = acc[1 + D + a][j]; }
          act_fwd<ACT, D>(z, pp, ee, av, Dv, Ev);
          float vals[7];
          vals[0] = av;
          for (int a = 0; a < D; ++a) { vals[1 + a] = Dv[a]; vals[1 + D + a] = Ev[a]; }
          Z[l - 2][0][j] = z;
          for (int s = 1; s < S; ++s) Z[l - 2][s][j] = acc[s][j];
          if (!last) {
            for (int s = 0; s < S; ++s) {
              T v = from_f<T>(vals[s]);
              bufR[cur ^ 1][s][c][n] = v;
              colA[l - 1][s][n][c] = v;
            }
          } else {
            for (int s = 0; s < S; ++s) colL[s][n][c] = vals[s];
          }
        }
        __syncthreads();
        cur ^= 1;
      }

      // ---------------- output layer and residual / adjoints
      for (int s = 0; s < S; ++s)
        for (int j = 0; j < 4; ++j) {
          float v = won * colL[s][n][4 * g + j];
          v += __shfl_xor(v, 8);
          v += __shfl_xor(v, 4);
          v += __shfl_xor(v, 2);
          v += __shfl_xor(v, 1);
          if (r16 == 0) part[w][4 * g + j][s] = v;
        }
      __syncthreads();
      __shared__ float ftile[kTile];
      if (inl && fpre) {
        if (tid < kTile) ftile[tid] = fpre[src[slot0 + tid]];
      } else if (inl && P.kind == 2) {
        // Fourier forcing: all threads, scratch in the (free) second row buffer
        tile_fourier<D, 256>(P, xs, reinterpret_cast<float*>(&bufR[1][0][0][0]), ftile);
      } else if (inl && tid < kTile) {
        float x[3] = {xs[tid][0], xs[tid][1], xs[tid][2]};
        ftile[tid] = f_side<float, D>(P, net, x);
      }
      __syncthreads();
      if (tid < kTile) {
        const int c = tid;
        const int64_t slot = slot0 + c;
        if (inl) {
          float eu = 0.f;
          for (int a = 0; a < D; ++a)
            for (int v = 0; v < 4; ++v) eu += part[v][c][1 + D + a];
          float r = -eu / hh - ftile[c] / (float)P.mu[net];
          resid[src[slot]] = r;
          lsum[c] += (double)r * (double)r;
          float rb = (float)(scale * (double)r);
          for (int s = 0; s < 8; ++s) adjs[c][s] = 0.f;
          for (int a = 0; a < D; ++a) adjs[c][1 + D + a] = -rb / hh;
        } else {
          const bool valid = slot < slot_end;
          for (int s = 0; s < 8; ++s) adjs[c][s] = valid ? adj[slot * 8 + s] : 0.f;
        }
      }
      __syncthreads();

      // ---------------- backward, top layer
      float dz[S][4];
      for (int j = 0; j < 4; ++j) {
        const int c = 4 * g + j;
        float pp[3], ee[3], Db[3], Eb[3], zb, pb[3], eb[3];
        for (int a = 0; a < D; ++a) {
          pp[a] = Z[L - 2][1 + a][j]; ee[a] = Z[L - 2][1 + D + a][j];
          Db[a] = won * adjs[c][1 + a]; Eb[a] = won * adjs[c][1 + D + a];
        }
        act_bwd<ACT, D>(Z[L - 2][0][j], pp, ee, won * adjs[c][0], Db, Eb, zb, pb, eb);
        dz[0][j] = zb;
        for (int a = 0; a < D; ++a) { dz[1 + a][j] = pb[a]; dz[1 + D + a][j] = eb[a]; }
        for (int s = 0; s < S; ++s) accwo += adjs[c][s] * colL[s][n][c];
      }
      if (tid == 0)
        for (int c = 0; c < kTile; ++c) accbo += adjs[c][0];

      // ---------------- backward through the hidden layers.  Per layer: dZ_l
      // goes to LDS in row layout, dA = dZ_l W_l runs on MFMA, then the dW_l
      // MFMAs (independent of dA) are issued next to the VALU derivative
      // epilogue of layer l-1 so that the two can overlap.
#pragma unroll
      for (int l = L; l >= 2; --l) {
        for (int j = 0; j < 4; ++j) accb[l - 1] += dz[0][j];
        for (int s = 0; s < S; ++s)
          for (int j = 0; j < 4; ++j) bufR[0][s][4 * g + j][n] = from_f<T>(dz[s][j]);
        __syncthreads();
        f4 acc[S];
        for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == 0) {
          float bk[KC];
          const float4* wp = (const float4*)((const float*)np.WlT[l - 2] + (int64_t)n * W + g * KC);
          for (int q = 0; q < KC / 4; ++q) {
            float4 v4 = wp[q];
            bk[4 * q] = v4.x; bk[4 * q + 1] = v4.y; bk[4 * q + 2] = v4.z; bk[4 * q + 3] = v4.w;
          }
          for (int s = 0; s < S; ++s) {
            const float4* ap = (const float4*)(&bufR[0][s][r16][g * KC]);
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
          const bf8* wp = (const bf8*)((const T*)np.WlT[l - 2] + (int64_t)n * W + g * KC);
          for (int q = 0; q < KC / 8; ++q) bk[q] = wp[q];
          for (int s = 0; s < S; ++s) {
            const bf8* ap = (const bf8*)(&bufR[0][s][r16][g * KC]);
            for (int q = 0; q < KC / 8; ++q) acc[s] = mfma32(ap[q], bk[q], acc[s]);
          }
        }
        // dW_l[n][:] += sum over (stream, centre) of dZ_l[.][n] A_{l-1}[.][:]
        for (int ib = 0; ib < NOB; ++ib) {
          const int nin = ib * 16 + r16;
          if constexpr (PREC == 0) {
            for (int s = 0; s < S; ++s) {
              float4 v = *(const float4*)(&colA[l - 2][s][nin][4 * g]);
              accW[l - 2][ib] = mfma4(dz[s][0], v.x, accW[l - 2][ib]);
              accW[l - 2][ib] = mfma4(dz[s][1], v.y, accW[l - 2][ib]);
              accW[l - 2][ib] = mfma4(dz[s][2], v.z, accW[l - 2][ib]);
              accW[l - 2][ib] = mfma4(dz[s][3], v.w, accW[l - 2][ib]);
            }
          } else {
            for (int s = 0; s < S; s += 2) {
              bf4 v0 = *(const bf4*)(&colA[l - 2][s][nin][4 * g]);
              bf4 v1 = (s + 1 < S) ? *(const bf4*)(&colA[l - 2][s + 1][nin][4 * g])
                                   : bf4{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
              bf8 av, bv;
              for (int j = 0; j < 4; ++j) {
                av[j] = (__bf16)dz[s][j];
                av[4 + j] = (s + 1 < S) ? (__bf16)dz[s + 1][j] : (__bf16)0.f;
                bv[j] = v0[j];
                bv[4 + j] = v1[j];
              }
              accW[l - 2][ib] = mfma32(av, bv, accW[l - 2][ib]);
            }
          }
        }
        // derivative epilogue of layer l-1 (pre-activations kept in registers)
        for (int j = 0; j < 4; ++j) {
          float pp[3], ee[3], Db[3], Eb[3], zb, pb[3], eb[3];
          if (l > 2) {
            for (int a = 0; a < D; ++a) {
              pp[a] = Z[l - 3][1 + a][j]; ee[a] = Z[l - 3][1 + D + a][j];
              Db[a] = acc[1 + a][j]; Eb[a] = acc[1 + D + a][j];
            }
            act_bwd<ACT, D>(Z[l - 3][0][j], pp, ee, acc[0][j], Db, Eb, zb, pb, eb);
            dz[0][j] = zb;
            for (int a = 0; a < D; ++a) { dz[1 + a][j] = pb[a]; dz[1 + D + a][j] = eb[a]; }
          } else {
            for (int a = 0; a < D; ++a) { Db[a] = acc[1 + a][j]; Eb[a] = acc[1 + D + a][j]; }
            act_bwd<ACT, D>(z1[j], p1, e0, acc[0][j], Db, Eb, zb, pb, eb);
            const int c = 4 * g + j;
            accb[0] += zb;
            for (int a = 0; a < D; ++a) accW1[a] += zb * xs[c][a] + h * pb[a];
          }
        }
        __syncthreads();   // bufR[0] is rewritten by the next layer
      }
    }

    // ---------------- flush this net's partial gradient
    float* prow = partial + (int64_t)blockIdx.x * Ptot + (net == 0 ? 0 : net_off1);
    for (int l = 2; l <= L; ++l)
      for (int ib = 0; ib < NOB; ++ib)
        for (int r = 0; r < 4; ++r) {
          int row = w * 16 + 4 * g + r, col = ib * 16 + r16;
          prow[lay.Wl[l - 2] + (int64_t)row * W + col] = accW[l - 2][ib][r];
        }
    for (int l = 0; l < L; ++l) {
      float v = accb[l];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      accb[l] = v;
    }
    float vwo = accwo;
    vwo += __shfl_xor(vwo, 16);
    vwo += __shfl_xor(vwo, 32);
    for (int a = 0; a < 3; ++a) {
      accW1[a] += __shfl_xor(accW1[a], 16);
      accW1[a] += __shfl_xor(accW1[a], 32);
    }
    if (g == 0) {
      prow[lay.b1 + n] = accb[0];
      for (int a = 0; a < D; ++a) prow[lay.W1 + (int64_t)n * D + a] = accW1[a];
      for (int l = 2; l <= L; ++l) prow[lay.bl[l - 2] + n] = accb[l - 1];
      prow[lay.wout + n] = vwo;
    }
    if (tid == 0) prow[lay.bout] = accbo;
    __syncthreads();
  }
  if (tid == 0) {
    double s = 0.0;
    for (int c = 0; c < kTile; ++c) s += lsum[c];
    lossp[blockIdx.x] = s;
  }
}

template <int D, int W, int L, int ACT, int PREC>
hipError_t fused_impl(const FusedCall& c) {
  hipLaunchKernelGGL((k_fused<D, W, L, ACT, PREC>), dim3(c.grid), dim3(256), 0, c.stream, c.meta,
                     c.centres, c.src, *c.nets, c.P, c.h, c.adj, c.resid, c.partial, c.Ptot, *c.lay,
                     c.off1, c.lossp, c.scale, c.fpre);
  return hipGetLastError();
}

#define NBM_FUSED(D, W, L, ACT, PREC) \
  if (dim == D && width == W && depth == L && act == ACT && prec == PREC) return &fused_impl<D, W, L, ACT, PREC>;

FusedFn find_fused(int dim, int width, int depth, int act, int prec) {
  NBM_FUSED(3, 64, 3, 0, 0)
  NBM_FUSED(3, 64, 3, 1, 0)
  NBM_FUSED(3, 64, 3, 0, 1)
  NBM_FUSED(3, 64, 3, 1, 1)
  return nullptr;
}

}  // namespace nbm
