// Fused forward + residual + backward over difference streams for W = 64
// networks.  A persistent work-group of four wavefronts walks 16-centre tiles;
// two work-groups share a compute unit so that the matrix-core phase of one
// overlaps the vector (activation) phase of the other.  Nothing per layer
// touches HBM:
//   * pre-activations (z and the difference streams) stay in registers
//     (FP32: parked in a dead row buffer between forward and backward);
//   * the GEMM operands of the current layer sit in LDS in row layout
//     [stream][centre][neuron], double-buffered between layers;
//   * activations of the hidden layers are not stored: the backward pass
//     recomputes them from the kept pre-activations while the matrix cores
//     form dA = dZ W, and dW^T = A^T dZ then takes A from registers and dZ
//     from LDS; dW accumulates in MFMA accumulators over all tiles.
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
__global__ __launch_bounds__(256, 2) void k_fused(const Meta* meta, const float4* centres, const int* src,
                                                  Nets nets, Problem P, float h, const float* adj,
                                                  float* resid, float* partial, int64_t Ptot,
                                                  NetLayout lay, int64_t net_off1, double* lossp,
                                                  double scale, const float* fslot) {
  typedef typename Op<PREC>::T T;
  constexpr int S = 2 * D + 1;
  constexpr int LD = W + (PREC == 0 ? 4 : 8);
  constexpr int NOB = W / 16;       // 16-neuron blocks; wave w owns block w
  constexpr int KC = W / 4;         // K chunk per lane group
  static_assert(NOB == 4, "one 16-neuron block per wave");
  // hidden layers with BF16 operands take the micro forms up to 1/32
  constexpr int kMicroL = PREC == 1 ? 2 : 0;
  __shared__ __attribute__((aligned(16))) T bufR[2][S][kTile][LD];      // row layout [c][n]
  // BF16 only: dZ also as [neuron][centre][stream (7 + zero)], the dW operand
  // (8 K values per lane = the streams of one centre); the odd centre stride
  // spreads the 16 neurons of a read over the banks
  constexpr bool kColZ = PREC == 1;
  __shared__ __attribute__((aligned(16))) T colZ[2][kColZ ? W : 1][kColZ ? kTile + 1 : 1][8];
  __shared__ float part[NOB][kTile][2];   // per wave: w_out . sum_i E_i of each centre
  __shared__ float adjs[kTile][8];
  __shared__ float xs[2][kTile][4];   // by tile parity
  __shared__ L1Axes l1ax[W];
  __shared__ double lsum[kTile];
  __shared__ int tflag;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, g = lane >> 4;
  const int n = w * 16 + r16;   // neuron owned by this lane, centres 4g..4g+3
  const int G = gridDim.x;
  const int ntiles = meta->tiles[0] + meta->tiles[1];
  const float hh = h * h;
  if (tid < kTile) lsum[tid] = 0.0;
  // this lane's B operand of one layer: row n of W_l (forward) or W_l^T
  // (backward), K chunk g; loaded one phase ahead of its MFMAs
  struct WRow { float f[PREC == 0 ? KC : 1]; bf8 b[PREC == 1 ? KC / 8 : 1]; };
  // wo: byte offset of the row segment, re-declared opaque on every tile so
  // the loads address memory as a scalar base plus a 32-bit lane offset
  // rather than through per-lane 64-bit addresses hoisted per matrix
  const uint32_t woff = (uint32_t)((n * W + g * KC) * (int)sizeof(T));
  auto load_w = [&](const void* m, uint32_t wo) {
    WRow r;
    if constexpr (PREC == 0) {
      const float4* wp = (const float4*)((const char*)m + wo);
      for (int q = 0; q < KC / 4; ++q) {
        float4 v4 = wp[q];
        r.f[4 * q] = v4.x; r.f[4 * q + 1] = v4.y; r.f[4 * q + 2] = v4.z; r.f[4 * q + 3] = v4.w;
      }
    } else {
      const bf8* wp = (const bf8*)((const char*)m + wo);
      for (int q = 0; q < KC / 8; ++q) r.b[q] = wp[q];
    }
    return r;
  };

  for (int net = 0; net < 2; ++net) {
    const NetPtrs& np = nets.net[net];
    f4 accW[L - 1][NOB];   // dW_l^T blocks: rows = inputs of block w, cols = outputs of block ob
    float accb[L], accW1[3] = {0.f, 0.f, 0.f}, accwo = 0.f, accbo = 0.f;
    for (int l = 0; l < L - 1; ++l)
      for (int k = 0; k < NOB; ++k) accW[l][k] = f4{0.f, 0.f, 0.f, 0.f};
    for (int l = 0; l < L; ++l) accb[l] = 0.f;
    float W1n[3], p1[3];
    for (int a = 0; a < D; ++a) { W1n[a] = np.W1[n * D + a]; p1[a] = h * W1n[a]; }
    // first-layer axis factors, constant per net: kept in LDS, not registers
    // micro first layer when every neuron of this wavefront has |h W1| <= 1/256
    const bool l1m = __all(l1_micro<D>(p1));
    if (g == 0) l1ax[n] = l1m ? l1_axes_micro<D>(p1) : l1_axes<ACT, D>(p1);
    __syncthreads();
    const float b1n = np.b1[n], won = np.wout[n];
    const float inv_hh = 1.0f / hh, inv_mu = 1.0f / (float)P.mu[net];
    const float kal = (float)(-scale / (double)hh);   // alpha_c = kal * r_c
    // Helmholtz term k u of the uncut residual, r += (k/mu) u: the base stream's
    // adjoint is alpha_c * rho with rho = -h^2 k/mu (zero without the term)
    const bool helm = P.kc[net] != 0.0;
    const float kmu = (float)(P.kc[net] / P.mu[net]), rho = -hh * kmu, bon = np.bout[0];
    const int64_t a_end = (int64_t)meta->base[net][KIND_A] + meta->cnt[net][KIND_A];
    const int t_lo = net == 0 ? 0 : meta->tiles[0];
    const int t_hi = net == 0 ? meta->tiles[0] : ntiles;

    const int64_t slot_end = (int64_t)meta->tile0[net] * kTile + meta->total[net];
    // per-tile global data (centres; forcing of inline tiles; adjoint rows of
    // the others) is fetched one tile ahead, so its latency hides behind the
    // current tile's work
    float4 nx = make_float4(0.f, 0.f, 0.f, 0.f);
    float nf = 0.f, na = 0.f;
    int ns = 0;
    auto fetch = [&](int tt) {
      const int64_t s0 = (int64_t)tt * kTile;
      if (tt >= t_hi) return;
      if (tid < kTile) {
        nx = s0 + tid < slot_end ? centres[s0 + tid] : make_float4(0.f, 0.f, 0.f, 0.f);
        if (s0 + kTile <= a_end) { nf = fslot[s0 + tid]; ns = src[s0 + tid]; }
      }
      if (s0 + kTile > a_end && tid < kTile * 8) na = s0 + tid / 8 < slot_end ? adj[s0 * 8 + tid] : 0.f;
    };
    fetch(t_lo + blockIdx.x);

    // Between tiles only xs and adjs are written before the first barrier of
    // the next tile (the row buffers after it).  xs alternates with the tile
    // parity X, since the last backward layer still reads it; adjs is last
    // read before the backward's first barrier.  So one barrier per tile
    // boundary suffices.
    int X = 0;
    for (int t = t_lo + blockIdx.x; t < t_hi; t += G) {
      const int64_t slot0 = (int64_t)t * kTile;
      const bool inl = slot0 + kTile <= a_end;   // uniform over the work-group
      // xs[c][3]: forcing of an inline tile's centre c (every wave forms the
      // residual of the centres it holds, so no wave waits for another's)
      if (tid < kTile) { xs[X][tid][0] = nx.x; xs[X][tid][1] = nx.y; xs[X][tid][2] = nx.z; xs[X][tid][3] = nf; }
      // output adjoints of a non-inline tile, written by the residual kernels
      if (!inl && tid < kTile * 8) adjs[tid / 8][tid % 8] = na;
      const int scur = ns;   // point index of this lane's centre (inline tiles)
      fetch(t + G);
      uint32_t wo = woff;
      asm volatile("" : "+v"(wo));
      __syncthreads();

      // ---------------- forward, layer 1 (VALU, accumulator mapping)
      float z1[4];
      for (int j = 0; j < 4; ++j) {
        const int c = 4 * g + j;
        float z = b1n;
        for (int a = 0; a < D; ++a) z += W1n[a] * xs[X][c][a];
        z1[j] = z;
        float av, Dv[3], Ev[3];
        act_fwd_l1_any<ACT, D>(l1m, z, l1ax[n], av, Dv, Ev);
        bufR[0][0][c][n] = from_f<T>(av);
        for (int a = 0; a < D; ++a) {
          bufR[0][1 + a][c][n] = from_f<T>(Dv[a]);
          bufR[0][1 + D + a][c][n] = from_f<T>(Ev[a]);
        }
      }
      WRow wn = load_w(np.Wl[0], wo);
      __syncthreads();

      // ---------------- forward, hidden layers on MFMA
      // pre-activations of layers 2..L-1 for (centres 4g+j, neuron n); the
      // last layer's backward is formed in its forward epilogue instead
      // FP32, three layers: once every wave is past the barrier that ends
      // layer 2, row buffer 0 (A_1) is dead until the next tile, so each
      // lane parks its layer-2 pre-activations there, in the slots
      // [s][4g+j][n] it alone reads back and later overwrites with dZ_2;
      // the backward's dZ_3 then uses buffer 1 (A_2 is dead after layer 3)
      constexpr bool kZlds = PREC == 0 && L == 3;
      float Z[L > 2 ? L - 2 : 1][S][4];
      float dz[S][4];         // dZ of the layer being differentiated
      float eS[4];            // last layer, inline tiles: sum over axes of the E streams
      int cur = 0;
#pragma unroll
      for (int l = 2; l <= L; ++l) {
        f4 acc[S];
        for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
        const WRow wcur = wn;
        mfma_phase_begin();
        if constexpr (PREC == 0) {
          for (int s = 0; s < S; ++s) {
            const float4* ap = (const float4*)(&bufR[cur][s][r16][g * KC]);
            for (int q = 0; q < KC / 4; ++q) {
              float4 a4 = ap[q];
              acc[s] = mfma4(a4.x, wcur.f[4 * q], acc[s]);
              acc[s] = mfma4(a4.y, wcur.f[4 * q + 1], acc[s]);
              acc[s] = mfma4(a4.z, wcur.f[4 * q + 2], acc[s]);
              acc[s] = mfma4(a4.w, wcur.f[4 * q + 3], acc[s]);
            }
          }
        } else {
          for (int s = 0; s < S; ++s) {
            const bf8* ap = (const bf8*)(&bufR[cur][s][r16][g * KC]);
            for (int q = 0; q < KC / 8; ++q) acc[s] = mfma32(ap[q], wcur.b[q], acc[s]);
          }
        }
        mfma_phase_end();
        const float bias = np.bl[l - 2][n];
        const bool last = (l == L);
        for (int j = 0; j < 4; ++j) {
          const int c = 4 * g + j;
          float z = acc[0][j] + bias;
          float pp[3], ee[3], av, Dv[3], Ev[3];
          for (int a = 0; a < D; ++a) { pp[a] = acc[1 + a][j]; ee[a] = acc[1 + D + a][j]; }
          if (!last) {
            act_fwd<ACT, D, kMicroL>(z, pp, ee, av, Dv, Ev);
            Z[l - 2][0][j] = z;
            for (int s = 1; s < S; ++s) Z[l - 2][s][j] = acc[s][j];
            bufR[cur ^ 1][0][c][n] = from_f<T>(av);
            for (int a = 0; a < D; ++a) {
              bufR[cur ^ 1][1 + a][c][n] = from_f<T>(Dv[a]);
              bufR[cur ^ 1][1 + D + a][c][n] = from_f<T>(Ev[a]);
            }
          } else {
            // output adjoints: known for non-inline tiles; inline tiles carry
            // one adjoint alpha_c on every E stream, known after the residual,
            // and the backward is linear in it: differentiate for w_out and
            // scale by alpha_c afterwards
            float ab, Db[3], Eb[3], zb, pb[3], eb[3];
            if (inl) {
              ab = rho * won;
              for (int a = 0; a < D; ++a) { Db[a] = 0.f; Eb[a] = won; }
            } else {
              ab = won * adjs[c][0];
              for (int a = 0; a < D; ++a) { Db[a] = won * adjs[c][1 + a]; Eb[a] = won * adjs[c][1 + D + a]; }
            }
            act_fb<ACT, D, kMicroL>(z, pp, ee, ab, Db, Eb, av, Dv, Ev, zb, pb, eb);
            dz[0][j] = zb;
            for (int a = 0; a < D; ++a) { dz[1 + a][j] = pb[a]; dz[1 + D + a][j] = eb[a]; }
            // output layer, u = sum_n w_out[n] a_L[n] (+ b_out) per stream: the
            // inline residual needs only sum_i eu_i, so this wave's share is one
            // reduction over its 16 neurons of w_out * sum_i E_i (non-inline
            // tiles take their outputs from the forward-only pass).
            // d loss / d w_out[n] = sum_c sum_s adj[c][s] a_L[s][n][c]
            if (inl) {
              float es = 0.f;
              for (int a = 0; a < D; ++a) es += Ev[a];
              // d loss / d w_out[n] of inline tiles: alpha_c (sum_i E_i + rho a)
              eS[j] = helm ? fmaf(rho, av, es) : es;
              const float v = row16_sum(won * es);
              if (r16 == 0) part[w][c][0] = v;
              if (helm) {
                const float vu = row16_sum(won * av);
                if (r16 == 0) part[w][c][1] = vu;
              }
            } else {
              accwo += adjs[c][0] * av;
              for (int a = 0; a < D; ++a) accwo += adjs[c][1 + a] * Dv[a];
              for (int a = 0; a < D; ++a) accwo += adjs[c][1 + D + a] * Ev[a];
            }
          }
        }
        // next phase's weights: the following layer, or the first backward layer
        wn = load_w(l < L ? np.Wl[l - 1] : np.WlT[L - 2], wo);
        __syncthreads();
        if (kZlds && l == 2)
          for (int s = 0; s < S; ++s)
            for (int j = 0; j < 4; ++j) bufR[0][s][4 * g + j][n] = Z[0][s][j];
        cur ^= 1;
      }

      // ---------------- residual / adjoints of inline tiles: the uncut
      // residual of centre c from the second-difference sums of the four
      // waves, and its adjoint alpha_c on every E stream.  Each lane forms
      // it for its own centres (same order everywhere, so the same value);
      // the first 16 lanes also store the residual and the loss term.
      auto uncut_r = [&](int c) {
        float eu = 0.f;
        for (int v = 0; v < NOB; ++v) eu += part[v][c][0];
        float r = -eu * inv_hh - xs[X][c][3] * inv_mu;
        if (helm) {
          float u = bon;
          for (int v = 0; v < NOB; ++v) u += part[v][c][1];
          r = fmaf(kmu, u, r);
        }
        return r;
      };
      if (inl) {
        if (tid < kTile) {
          const float r = uncut_r(tid);
          resid[scur] = r;
          lsum[tid] += (double)r * (double)r;
        }
        // top layer of inline tiles: scale by alpha_c = d loss / d eu_c
        for (int j = 0; j < 4; ++j) {
          const float al = kal * uncut_r(4 * g + j);
          for (int s = 0; s < S; ++s) dz[s][j] *= al;
          accwo += al * eS[j];
        }
        // d loss / d b_out = sum_c alpha_c rho (zero without the k term)
        if (helm && tid == 0)
          for (int c = 0; c < kTile; ++c) accbo += rho * kal * uncut_r(c);
      } else if (tid == 0) {
        for (int c = 0; c < kTile; ++c) accbo += adjs[c][0];
      }

      // ---------------- backward through the hidden layers.  Per layer l:
      // dZ_l goes to LDS; dA_{l-1} = dZ_l W_l runs on the matrix cores; then
      // per centre the VALU recomputes A_{l-1} and forms dZ_{l-1}, and the
      // dW_l^T = A_{l-1}^T dZ_l MFMAs consume A_{l-1}.
      int bb = kZlds ? 1 : 0;
#pragma unroll
      for (int l = L; l >= 2; --l) {
        for (int j = 0; j < 4; ++j) accb[l - 1] += dz[0][j];
        for (int s = 0; s < S; ++s)
          for (int j = 0; j < 4; ++j) bufR[bb][s][4 * g + j][n] = from_f<T>(dz[s][j]);
        if constexpr (kColZ) {
          for (int j = 0; j < 4; ++j) {
            bf8 v;
            for (int k = 0; k < S; ++k) v[k] = (__bf16)dz[k][j];
            for (int k = S; k < 8; ++k) v[k] = (__bf16)0.f;
            *(bf8*)(&colZ[bb][n][4 * g + j][0]) = v;
          }
        }
        __syncthreads();
        f4 acc[S];
        for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
        const WRow wcur = wn;
        if (l > 2) wn = load_w(np.WlT[l - 3], wo);   // next backward layer's weights
        mfma_phase_begin();
        if constexpr (PREC == 0) {
          for (int s = 0; s < S; ++s) {
            const float4* ap = (const float4*)(&bufR[bb][s][r16][g * KC]);
            for (int q = 0; q < KC / 4; ++q) {
              float4 a4 = ap[q];
              acc[s] = mfma4(a4.x, wcur.f[4 * q], acc[s]);
              acc[s] = mfma4(a4.y, wcur.f[4 * q + 1], acc[s]);
              acc[s] = mfma4(a4.z, wcur.f[4 * q + 2], acc[s]);
              acc[s] = mfma4(a4.w, wcur.f[4 * q + 3], acc[s]);
            }
          }
        } else {
          for (int s = 0; s < S; ++s) {
            const bf8* ap = (const bf8*)(&bufR[bb][s][r16][g * KC]);
            for (int q = 0; q < KC / 8; ++q) acc[s] = mfma32(ap[q], wcur.b[q], acc[s]);
          }
        }
        mfma_phase_end();
        // per centre j: A_{l-1} recomputed from its pre-activations (layer 1:
        // from z1) together with the derivative epilogue dZ_{l-1}, sharing
        // the activation factors; then dW_l^T[n_in][n_out] += sum over
        // streams of A[.][n_in] dZ_l[.][n_out]
        for (int j = 0; j < 4; ++j) {
          float av[S], Dv[3], Ev[3], Db[3], Eb[3], zb, pb[3], eb[3];
          for (int a = 0; a < D; ++a) { Db[a] = acc[1 + a][j]; Eb[a] = acc[1 + D + a][j]; }
          if (l > 2) {
            float zz, pp[3], ee[3];
            if constexpr (kZlds) {
              const int c = 4 * g + j;
              zz = bufR[0][0][c][n];
              for (int a = 0; a < D; ++a) { pp[a] = bufR[0][1 + a][c][n]; ee[a] = bufR[0][1 + D + a][c][n]; }
            } else {
              zz = Z[l - 3][0][j];
              for (int a = 0; a < D; ++a) { pp[a] = Z[l - 3][1 + a][j]; ee[a] = Z[l - 3][1 + D + a][j]; }
            }
            act_fb<ACT, D, kMicroL>(zz, pp, ee, acc[0][j], Db, Eb, av[0], Dv, Ev, zb, pb, eb);
          } else {
            act_fb_l1_any<ACT, D>(l1m, z1[j], l1ax[n], acc[0][j], Db, Eb, av[0], Dv, Ev, zb, pb);
          }
          for (int a = 0; a < D; ++a) { av[1 + a] = Dv[a]; av[1 + D + a] = Ev[a]; }
          if constexpr (PREC == 0) {
            for (int ob = 0; ob < NOB; ++ob)
              for (int s = 0; s < S; ++s)
                accW[l - 2][ob] = mfma4(av[s], bufR[bb][s][4 * g + j][ob * 16 + r16], accW[l - 2][ob]);
          } else {
            // K = 8 per MFMA: the seven streams of centre 4g+j and a zero
            bf8 aop;
            for (int k = 0; k < S; ++k) aop[k] = (__bf16)av[k];
            for (int k = S; k < 8; ++k) aop[k] = (__bf16)0.f;
            for (int ob = 0; ob < NOB; ++ob) {
              const bf8 bop = *(const bf8*)(&colZ[bb][ob * 16 + r16][4 * g + j][0]);
              accW[l - 2][ob] = mfma32(aop, bop, accW[l - 2][ob]);
            }
          }
          if (l > 2) {
            dz[0][j] = zb;
            for (int a = 0; a < D; ++a) { dz[1 + a][j] = pb[a]; dz[1 + D + a][j] = eb[a]; }
          } else {
            const int c = 4 * g + j;
            accb[0] += zb;
            for (int a = 0; a < D; ++a) accW1[a] += zb * xs[X][c][a] + h * pb[a];
          }
        }
        bb ^= 1;   // the other row buffer: no barrier needed before the next write
      }
      X ^= 1;
    }

    // ---------------- flush this net's partial gradient
    float* prow = partial + (int64_t)blockIdx.x * Ptot + (net == 0 ? 0 : net_off1);
    for (int l = 2; l <= L; ++l)
      for (int ob = 0; ob < NOB; ++ob)
        for (int r = 0; r < 4; ++r) {
          const int nin = w * 16 + 4 * g + r, nout = ob * 16 + r16;
          prow[lay.Wl[l - 2] + (int64_t)nout * W + nin] = accW[l - 2][ob][r];
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
                     c.off1, c.lossp, c.scale, c.fslot);
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
