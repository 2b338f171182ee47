// Training step for W = 128 networks in two passes.
//
// Pass 1 (k_wide_fb): one persistent work-group of W/16 wavefronts per
// 16-centre tile walks forward through every layer (pre-activations stay in
// registers: each lane owns one neuron and four centres), forms the last
// layer's backward in its forward epilogue, the uncut residual inline (or
// takes the adjoints written by the residual kernels for other tiles), and
// walks backward computing dZ_l for every hidden layer.
// The operands of the weight-gradient contraction, A_{l-1} and dZ_l, leave
// the chip in the accumulator ("tile") layout [tile][stream][neuron][16]
// (with BF16 operands except A_1, which pass 2 rebuilds from the centres);
// the small gradients (biases, W_1, w_out) are accumulated per work-group.
// Loads and stores retire through one counter, so loads are placed ahead of
// the store bursts they would otherwise wait behind.  The operand rows cross
// HBM once (written here, read once by pass 2), so both sides use streaming
// (non-temporal) accesses and leave the caches to the reused data.
//
// With BF16 operands the forward/backward pass runs first in a fast form
// that takes the micro tier of the activation streams for every element
// without branching (keeping the running maximum of the tier's arguments);
// if any argument lies beyond the tier's bound it raises meta->slow, and the
// general form, launched right after and otherwise exiting at once,
// recomputes the whole pass with per-element tiers, overwriting every output
// of the fast one.  FP32 operands run the general form alone.
//
// Pass 2 (k_wide_dw, nbm_wide_dw.hip): dW_l = sum over (tile, stream, centre) of dZ_l^T A_{l-1}
// read straight from the tile layout as MFMA operands (the K index runs over
// stream pairs x 4 centres per lane group), split over persistent work-groups
// that each write one partial row; the FP64 reduction follows.
#include <hip/hip_runtime.h>

#include "nbm_device.hpp"
#include "nbm_internal.hpp"
#include "nbm_launch.hpp"

namespace nbm {

template <int D, int W, int L, int ACT, int PREC, bool FAST>
__global__ __launch_bounds__(W * 4) void k_wide_fb(const Meta* meta, const float4* centres,
                                                   const int* src, Nets nets, Problem P, float h,
                                                   const float* adj, float* resid, void* Aout_,
                                                   void* dZout_, int64_t lstride, float* partial,
                                                   int64_t Ptot, NetLayout lay, int64_t net_off1,
                                                   double* lossp, double scale, const float* fslot,
                                                   int* slow) {
  typedef typename Op<PREC>::T T;
  // the general form runs only when the fast form flagged an argument (or
  // unconditionally, with slow = null, where no fast form precedes it)
  if constexpr (!FAST)
    if (slow != nullptr && *slow == 0) return;
  float amax = 0.f;   // fast form: largest micro argument this lane met
  constexpr int S = 2 * D + 1;
  constexpr int NW = W / 16;     // wavefronts; wave w owns neurons 16w .. 16w+15
  constexpr int KC = W / 4;
  // micro forms of the hidden layers: up to 1/256, or 1/32 with BF16 operands
  constexpr int kMicroW = PREC == 1 ? 2 : 1;
  // Row buffers of the 16 centres' activations (or adjoints), the A operand
  // of every product, double-buffered per stream.  BF16: chunk-major, the
  // 16-byte chunk k (neurons 8k .. 8k+7) of all 16 centres side by side, and
  // lane group g takes chunk 4q + g at product step q, so a wavefront's
  // operand read covers 1 KB in lane order (free of LDS bank conflicts,
  // where padded rows cost extra cycles on every read).  FP32: centre rows
  // padded to W + 4, lane group g taking neurons g W/4 + 4q .. + 3 at step q
  // (the chunk-major order measured slower there: its 32-bit row writes
  // conflict where the 16-bit ones of BF16 conflict less).
  constexpr int EPC = 16 / (int)sizeof(T);   // values per 16-byte chunk
  constexpr int kRowBuf = PREC == 1 ? kTile * W : kTile * (W + 4);
  __shared__ __attribute__((aligned(16))) T bufR[2][S][kRowBuf];
  // position of (centre c, neuron m) and of lane (r16, g)'s operand at step q
  auto rpos = [](int c, int m) {
    return PREC == 1 ? (m / EPC) * (kTile * EPC) + c * EPC + m % EPC : c * (W + 4) + m;
  };
  auto apos = [](int r, int gg, int q) {
    return PREC == 1 ? (4 * q + gg) * (kTile * EPC) + r * EPC : r * (W + 4) + gg * KC + 4 * q;
  };
  // BF16 operands leave room in LDS for the first hidden layer's
  // pre-activations [stream][neuron][centre] (each lane reads back only what
  // it wrote); FP32 operands keep them in registers
  constexpr bool kZ0inLDS = PREC == 1;
  // [stream][centre group g][neuron][4 centres]: a wavefront's float4 accesses are contiguous
  __shared__ __attribute__((aligned(16))) float Zs[kZ0inLDS ? S : 1][kZ0inLDS ? 4 : 1][kZ0inLDS ? W : 1][4];
  __shared__ float adjs[kTile][8];
  __shared__ float part[NW][kTile][2];   // per wave: w_out . sum_i E_i of each centre
  __shared__ float xs[kTile][4];
  __shared__ L1Axes l1ax[W];
  __shared__ double lsum[kTile];
  T* Aout = (T*)Aout_;
  T* dZout = (T*)dZout_;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, g = lane >> 4;
  const int n = w * 16 + r16;
  // byte offset of this lane's first weight operand in a W x W matrix (row n;
  // BF16: chunk g, then every fourth chunk, matching the row buffer's order)
  const uint32_t woff = (uint32_t)((n * W + g * (PREC == 1 ? EPC : KC)) * (int)sizeof(T));
  const int G = gridDim.x;
  const int ntiles = meta->tiles[0] + meta->tiles[1];
  const float hh = h * h;
  if (tid < kTile) lsum[tid] = 0.0;

  for (int net = 0; net < 2; ++net) {
    const NetPtrs& np = nets.net[net];
    float accb[L], accW1[3] = {0.f, 0.f, 0.f}, accwo = 0.f, accbo = 0.f;
    for (int l = 0; l < L; ++l) accb[l] = 0.f;
    float W1n[3], p1[3];
    for (int a = 0; a < D; ++a) { W1n[a] = np.W1[n * D + a]; p1[a] = h * W1n[a]; }
    // first-layer axis factors, constant per net: kept in LDS, not registers
    if (g == 0) l1ax[n] = l1_axes<ACT, D>(p1);
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
    // read once per net: inside the tile loop the batch record would be
    // re-read after every tile's stores (which the compiler cannot rule out
    // aliasing it), and that read would wait for them
    const int64_t slot_end = (int64_t)meta->tile0[net] * kTile + meta->total[net];

    for (int t = t_lo + blockIdx.x; t < t_hi; t += G) {
      const int64_t slot0 = (int64_t)t * kTile;
      const bool inl = slot0 + kTile <= a_end;   // uniform over the work-group
      if (tid < kTile) {
        float4 cc = centres[slot0 + tid];
        if (slot0 + tid >= slot_end) cc = make_float4(0.f, 0.f, 0.f, 0.f);
        // xs[c][3]: forcing of an inline tile's centre (every lane forms the
        // residual of the centres it holds)
        xs[tid][0] = cc.x; xs[tid][1] = cc.y; xs[tid][2] = cc.z;
        xs[tid][3] = inl ? fslot[slot0 + tid] : 0.f;
      }
      // point index of an inline tile's centre, read here with the centres:
      // a read at the residual would wait for the operand-row stores issued
      // before it
      const int scur = inl && tid < kTile ? src[slot0 + tid] : 0;
      if (!inl && tid < kTile * 8) {
        // output adjoints of a non-inline tile, written by the residual kernels
        const int64_t slot = slot0 + tid / 8;
        adjs[tid / 8][tid % 8] = slot < slot_end ? adj[slot0 * 8 + tid] : 0.f;
      }
      __syncthreads();
      // Operand rows of this tile: a wave-uniform base (the tile's block)
      // and a 32-bit per-lane offset, so the stores address memory as a
      // scalar base plus a vector offset instead of holding a 64-bit address
      // per lane and layer in registers
      // (the empty asm statements keep the compiler from folding the offsets
      // into per-lane 64-bit addresses hoisted out of the tile loop)
      uint32_t roff = (uint32_t)((n * kTile + 4 * g) * (int)sizeof(T));
      uint32_t wo = woff;
      asm volatile("" : "+v"(roff), "+v"(wo));
      auto rowp = [&](T* layer_base, int s) -> T* {
        T* tb = layer_base + (int64_t)t * S * W * kTile;
        return (T*)((char*)tb + (roff + (uint32_t)(s * W * kTile * (int)sizeof(T))));
      };

      // ---- layer 1
      float z1[4];
      for (int j = 0; j < 4; ++j) {
        const int c = 4 * g + j;
        float z = b1n;
        for (int a = 0; a < D; ++a) z += W1n[a] * xs[c][a];
        z1[j] = z;
      }
      {
        float vals[S][4];
        for (int j = 0; j < 4; ++j) {
          float av, Dv[3], Ev[3];
          act_fwd_l1<ACT, D>(z1[j], l1ax[n], av, Dv, Ev);
          vals[0][j] = av;
          for (int a = 0; a < D; ++a) { vals[1 + a][j] = Dv[a]; vals[1 + D + a][j] = Ev[a]; }
        }
        for (int s = 0; s < S; ++s) {
          for (int j = 0; j < 4; ++j) bufR[0][s][rpos(4 * g + j, n)] = from_f<T>(vals[s][j]);
          // first-layer operand rows: stored with FP32 operands; with BF16 the
          // weight-gradient pass rebuilds them from the centres
          if constexpr (PREC == 0)
            st_stream((float*)rowp(Aout, s), f4{vals[s][0], vals[s][1], vals[s][2], vals[s][3]});
        }
      }
      __syncthreads();

      // ---- hidden layers.  Pre-activations of layers 2..L-1 stay in
      // registers; the last layer's backward is formed in its epilogue.
      float Z[L - 2][S][4];
      float dz[S][4];
      float eS[4];
      int cur = 0;
      // BF16: this lane's weight operand of the next product, loaded just
      // before the operand-row stores that precede it (loads and stores retire
      // through one counter, so a load issued after the stores would wait for
      // them to reach memory)
      bf8 wk[PREC == 1 ? KC / 8 : 1];
      float wbias = 0.f;   // and the forward product's bias
      auto load_wk = [&](const void* m, const float* bias_row) {
        if constexpr (PREC == 1) {
          const bf8* wp = (const bf8*)((const char*)m + wo);
          for (int q = 0; q < KC / 8; ++q) wk[q] = wp[4 * q];
          if (bias_row != nullptr) wbias = bias_row[n];
        }
      };
      load_wk(np.Wl[0], np.bl[0]);
#pragma unroll
      for (int l = 2; l <= L; ++l) {
        f4 acc[S];
        for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
        mfma_phase_begin();
        if constexpr (PREC == 0) {
          const float4* wp = (const float4*)((const char*)np.Wl[l - 2] + wo);
          for (int q = 0; q < KC / 4; ++q) {
            float4 b4 = wp[q];
            for (int s = 0; s < S; ++s) {
              float4 a4 = *(const float4*)(&bufR[cur][s][apos(r16, g, q)]);
              acc[s] = mfma4(a4.x, b4.x, acc[s]);
              acc[s] = mfma4(a4.y, b4.y, acc[s]);
              acc[s] = mfma4(a4.z, b4.z, acc[s]);
              acc[s] = mfma4(a4.w, b4.w, acc[s]);
            }
          }
        } else {
          for (int q = 0; q < KC / 8; ++q)
            for (int s = 0; s < S; ++s) acc[s] = mfma32(*(const bf8*)(&bufR[cur][s][apos(r16, g, q)]), wk[q], acc[s]);
        }
        mfma_phase_end();
        const float bias = PREC == 1 ? wbias : np.bl[l - 2][n];
        if (l < L) {
          float vals[S][4];
          for (int j = 0; j < 4; ++j) {
            float z = acc[0][j] + bias;
            float pp[3], ee[3], av, Dv[3], Ev[3];
            for (int a = 0; a < D; ++a) { pp[a] = acc[1 + a][j]; ee[a] = acc[1 + D + a][j]; }
            if constexpr (FAST) {
              amax = fmaxf(amax, micro_extent<D>(pp, ee));
              act_fwd_micro<ACT, D, kMicroW>(z, pp, ee, av, Dv, Ev);
            } else {
              act_fwd<ACT, D, kMicroW>(z, pp, ee, av, Dv, Ev);
            }
            Z[l - 2][0][j] = z;
            for (int s = 1; s < S; ++s) Z[l - 2][s][j] = acc[s][j];
            vals[0][j] = av;
            for (int a = 0; a < D; ++a) { vals[1 + a][j] = Dv[a]; vals[1 + D + a][j] = Ev[a]; }
          }
          if (kZ0inLDS && l == 2)
            for (int s = 0; s < S; ++s)
              *(float4*)(&Zs[s][g][n][0]) = make_float4(Z[0][s][0], Z[0][s][1], Z[0][s][2], Z[0][s][3]);
          load_wk(np.Wl[l - 1], np.bl[l - 1]);   // the next layer's product
          for (int s = 0; s < S; ++s) {
            for (int j = 0; j < 4; ++j) bufR[cur ^ 1][s][rpos(4 * g + j, n)] = from_f<T>(vals[s][j]);
            T* dst = rowp(Aout + (int64_t)(l - 1) * lstride, s);
            if constexpr (PREC == 0)
              st_stream((float*)dst, f4{vals[s][0], vals[s][1], vals[s][2], vals[s][3]});
            else
              st_stream((bf4*)dst, bf4{(__bf16)vals[s][0], (__bf16)vals[s][1], (__bf16)vals[s][2], (__bf16)vals[s][3]});
          }
        } else {
          // output adjoints: known for non-inline tiles; inline tiles carry one
          // adjoint alpha_c on every E stream (known after the residual) and
          // the backward is linear in it
          for (int j = 0; j < 4; ++j) {
            const int c = 4 * g + j;
            float z = acc[0][j] + bias;
            float pp[3], ee[3], av, Dv[3], Ev[3], ab, Db[3], Eb[3], zb, pb[3], eb[3];
            for (int a = 0; a < D; ++a) { pp[a] = acc[1 + a][j]; ee[a] = acc[1 + D + a][j]; }
            if (inl) {
              ab = rho * won;
              for (int a = 0; a < D; ++a) { Db[a] = 0.f; Eb[a] = won; }
            } else {
              ab = won * adjs[c][0];
              for (int a = 0; a < D; ++a) { Db[a] = won * adjs[c][1 + a]; Eb[a] = won * adjs[c][1 + D + a]; }
            }
            if constexpr (FAST) {
              amax = fmaxf(amax, micro_extent<D>(pp, ee));
              act_fb_micro<ACT, D, kMicroW>(z, pp, ee, ab, Db, Eb, av, Dv, Ev, zb, pb, eb);
            } else {
              act_fb<ACT, D, kMicroW>(z, pp, ee, ab, Db, Eb, av, Dv, Ev, zb, pb, eb);
            }
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
        __syncthreads();
        cur ^= 1;
      }

      // ---- residual / adjoints of inline tiles: the uncut residual of centre
      // c from the waves' second-difference sums and its adjoint alpha_c on
      // every E stream, formed by each lane for its own centres (same order
      // everywhere, so the same value); the first 16 lanes also store the
      // residual and the loss term
      auto uncut_r = [&](int c) {
        float eu = 0.f;
        for (int v = 0; v < NW; ++v) eu += part[v][c][0];
        float r = -eu * inv_hh - xs[c][3] * inv_mu;
        if (helm) {
          float u = bon;
          for (int v = 0; v < NW; ++v) u += part[v][c][1];
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

      // ---- backward through the hidden layers (dZ rows double-buffered)
      int bb = 0;
#pragma unroll
      for (int l = L; l >= 2; --l) {
        for (int j = 0; j < 4; ++j) accb[l - 1] += dz[0][j];
        load_wk(np.WlT[l - 2], nullptr);   // this layer's transposed product, below
        for (int s = 0; s < S; ++s) {
          for (int j = 0; j < 4; ++j) bufR[bb][s][rpos(4 * g + j, n)] = from_f<T>(dz[s][j]);
          T* dst = rowp(dZout + (int64_t)(l - 2) * lstride, s);
          if constexpr (PREC == 0)
            st_stream((float*)dst, f4{dz[s][0], dz[s][1], dz[s][2], dz[s][3]});
          else
            st_stream((bf4*)dst, bf4{(__bf16)dz[s][0], (__bf16)dz[s][1], (__bf16)dz[s][2], (__bf16)dz[s][3]});
        }
        __syncthreads();
        f4 acc[S];
        for (int s = 0; s < S; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
        mfma_phase_begin();
        if constexpr (PREC == 0) {
          const float4* wp = (const float4*)((const char*)np.WlT[l - 2] + wo);
          for (int q = 0; q < KC / 4; ++q) {
            float4 b4 = wp[q];
            for (int s = 0; s < S; ++s) {
              float4 a4 = *(const float4*)(&bufR[bb][s][apos(r16, g, q)]);
              acc[s] = mfma4(a4.x, b4.x, acc[s]);
              acc[s] = mfma4(a4.y, b4.y, acc[s]);
              acc[s] = mfma4(a4.z, b4.z, acc[s]);
              acc[s] = mfma4(a4.w, b4.w, acc[s]);
            }
          }
        } else {
          for (int q = 0; q < KC / 8; ++q)
            for (int s = 0; s < S; ++s) acc[s] = mfma32(*(const bf8*)(&bufR[bb][s][apos(r16, g, q)]), wk[q], acc[s]);
        }
        mfma_phase_end();
        if (kZ0inLDS && l == 3)
          for (int s = 0; s < S; ++s) {
            const float4 v = *(const float4*)(&Zs[s][g][n][0]);
            Z[0][s][0] = v.x; Z[0][s][1] = v.y; Z[0][s][2] = v.z; Z[0][s][3] = v.w;
          }
        for (int j = 0; j < 4; ++j) {
          float pp[3], ee[3], Db[3], Eb[3], zb, pb[3], eb[3];
          for (int a = 0; a < D; ++a) { Db[a] = acc[1 + a][j]; Eb[a] = acc[1 + D + a][j]; }
          if (l > 2) {
            for (int a = 0; a < D; ++a) { pp[a] = Z[l - 3][1 + a][j]; ee[a] = Z[l - 3][1 + D + a][j]; }
            // (the same arguments as in the forward: the fast form checked them there)
            if constexpr (FAST) act_bwd_micro<ACT, D, kMicroW>(Z[l - 3][0][j], pp, ee, acc[0][j], Db, Eb, zb, pb, eb);
            else act_bwd<ACT, D, kMicroW>(Z[l - 3][0][j], pp, ee, acc[0][j], Db, Eb, zb, pb, eb);
            dz[0][j] = zb;
            for (int a = 0; a < D; ++a) { dz[1 + a][j] = pb[a]; dz[1 + D + a][j] = eb[a]; }
          } else {
            act_bwd_l1<ACT, D>(z1[j], l1ax[n], acc[0][j], Db, Eb, zb, pb);
            const int c = 4 * g + j;
            accb[0] += zb;
            for (int a = 0; a < D; ++a) accW1[a] += zb * xs[c][a] + h * pb[a];
          }
        }
        bb ^= 1;
      }
      __syncthreads();   // xs, adjs and the row buffers are rewritten by the next tile
    }
    // ---- flush the small gradients of this net
    float* prow = partial + (int64_t)blockIdx.x * Ptot + (net == 0 ? 0 : net_off1);
    for (int l = 0; l < L; ++l) {
      float v = accb[l];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      accb[l] = v;
    }
    accwo += __shfl_xor(accwo, 16);
    accwo += __shfl_xor(accwo, 32);
    for (int a = 0; a < 3; ++a) {
      accW1[a] += __shfl_xor(accW1[a], 16);
      accW1[a] += __shfl_xor(accW1[a], 32);
    }
    if (g == 0) {
      prow[lay.b1 + n] = accb[0];
      for (int a = 0; a < D; ++a) prow[lay.W1 + (int64_t)n * D + a] = accW1[a];
      for (int l = 2; l <= L; ++l) prow[lay.bl[l - 2] + n] = accb[l - 1];
      prow[lay.wout + n] = accwo;
    }
    if (tid == 0) prow[lay.bout] = accbo;
    __syncthreads();
  }
  if (tid == 0) {
    double s = 0.0;
    for (int c = 0; c < kTile; ++c) s += lsum[c];
    lossp[blockIdx.x] = s;
  }
  // (written so that a NaN argument also sends the pass to the general form)
  if constexpr (FAST)
    if (!(amax <= micro_bound<kMicroW>())) *slow = 1;
}

// pass 2, in nbm_wide_dw.hip: k_wide_dw for hidden layer l (2 .. L)
template <int D, int W, int PREC, int ACT>
hipError_t launch_wide_dw(const WideCall& c, int l);

template <int D, int W, int L, int ACT, int PREC>
hipError_t wide_impl(const WideCall& c) {
  // The fast form is used with BF16 operands, whose micro bound (1/32) the
  // arguments of trained networks stay within; with FP32 operands the bound
  // is 1/256, which trained weights leave, and a fast pass would then be
  // repeated by the general one every step, so FP32 runs the general form
  // alone.
  int* slow = PREC == 1 ? const_cast<int*>(&c.meta->slow) : nullptr;   // inside the batch record
  hipError_t e = hipSuccess;
  if constexpr (PREC == 1) {
    hipLaunchKernelGGL((k_wide_fb<D, W, L, ACT, PREC, true>), dim3(c.grid), dim3(W * 4), 0, c.stream,
                       c.meta, c.centres, c.src, *c.nets, c.P, c.h, c.adj, c.resid, c.A, c.dZ, c.lstride,
                       c.partial, c.Ptot, *c.lay, c.off1, c.lossp, c.scale, c.fslot, slow);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_wide_fb<D, W, L, ACT, PREC, false>), dim3(c.grid), dim3(W * 4), 0, c.stream,
                       c.meta, c.centres, c.src, *c.nets, c.P, c.h, c.adj, c.resid, c.A, c.dZ, c.lstride,
                       c.partial, c.Ptot, *c.lay, c.off1, c.lossp, c.scale, c.fslot, slow);
    e = hipGetLastError();
  }
  if (c.after_fb) c.after_fb(c.timer_ctx);
  if (e != hipSuccess) return e;
  for (int l = 2; l <= L; ++l) {
    if (c.timer_begin) c.timer_begin(c.timer_ctx);
    e = launch_wide_dw<D, W, PREC, ACT>(c, l);
    if (c.timer_end) c.timer_end(c.timer_ctx);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

#define NBM_WIDE(D, W, L, ACT, PREC) \
  if (dim == D && width == W && depth == L && act == ACT && prec == PREC) return &wide_impl<D, W, L, ACT, PREC>;

WideFn find_wide(int dim, int width, int depth, int act, int prec) {
  NBM_WIDE(3, 128, 4, 1, 1)
  NBM_WIDE(3, 128, 4, 1, 0)
  NBM_WIDE(3, 128, 4, 0, 1)
  NBM_WIDE(3, 128, 4, 0, 0)
  return nullptr;
}

}  // namespace nbm
