// Host-side launcher interface between the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "nbm_internal.hpp"

namespace nbm {

struct MlpCall {
  enum Op { FORWARD, BACKWARD } op;
  hipStream_t stream;
  int grid;
  const Meta* meta;
  const float4* centres;
  const Nets* nets;
  int L, l;
  float h;
  float* outputs;
  const float* adj;
  float* Zst;
  void* Ast;
  float* ALst;
  float* dZ;
  float* partial;
  int64_t Ptot;
  const NetLayout* lay;
  int64_t off1;
  int64_t lstride;
  bool store, streams;
  int noninline;
};
typedef hipError_t (*MlpFn)(const MlpCall&);
MlpFn find_mlp(int dim, int width, int act, int prec);

// base-stream forward of the evaluation path (persistent work-groups)
struct EvalCall {
  hipStream_t stream;
  int max_grid;              // upper bound on useful work-groups (tiles of 64 centres)
  const Meta* meta;
  const float4* centres;
  const int* src;
  const Nets* nets;
  float* u_out;              // [m], indexed by query
};
typedef hipError_t (*EvalFn)(const EvalCall&);
EvalFn find_eval(int dim, int width, int depth, int act, int prec);

struct FusedCall {
  const float* fslot;  // forcing of uncut centres in centre-slot order
  hipStream_t stream;
  int grid;
  const Meta* meta;
  const float4* centres;
  const int* src;
  const Nets* nets;
  Problem P;
  float h;
  const float* adj;
  float* resid;
  float* partial;
  int64_t Ptot;
  const NetLayout* lay;
  int64_t off1;
  double* lossp;
  double scale;
};
typedef hipError_t (*FusedFn)(const FusedCall&);
FusedFn find_fused(int dim, int width, int depth, int act, int prec);

struct WideCall {
  const float* fslot;  // forcing of uncut centres in centre-slot order
  hipStream_t stream;
  int grid;
  const Meta* meta;
  const float4* centres;
  const int* src;
  const Nets* nets;
  Problem P;
  float h;
  const float* adj;
  float* resid;
  void* A;       // (L-1) layers of activations, tile layout, operand dtype
  void* dZ;      // (L-1) layers of pre-activation adjoints, tile layout, operand dtype
  int64_t lstride;
  float* partial;
  int64_t Ptot;
  const NetLayout* lay;
  int64_t off1;
  double* lossp;
  double scale;
  void (*after_fb)(void*);      // called after the forward/backward launch (or null)
  void (*timer_begin)(void*);   // called around each weight-gradient launch (or null)
  void (*timer_end)(void*);
  void* timer_ctx;
};
typedef hipError_t (*WideFn)(const WideCall&);
WideFn find_wide(int dim, int width, int depth, int act, int prec);

// operand copies (W_l and W_l^T in the operand dtype) of up to 16 hidden
// matrices (two nets of depth <= 8), made by extra blocks of the classify launch
struct ShadowJobs {
  const float* params;
  int64_t off[16];
  void* Wl[16];
  void* WlT[16];
  int count;
  int W;
};

struct PrepCall {
  hipStream_t stream;
  Problem P;
  const float* pts;
  int64_t n;
  const float* bpts;
  int64_t nb;
  bool eval;
  int64_t tile_index;
  int grid_n;
  int cut_cap;
  int *cls, *rank, *blockcnt, *off;
  int *bcls, *brank, *blockcnt_b, *off_b;
  Meta* meta;
  float4* centres;
  int* src;
  int* cutidx;
  ShadowJobs shadows;   // operand copies made in the same launch (count 0: none)
  int prec;
  float* fslot;         // manufactured forcing of uncut points in slot order, or NULL
  // chunk totals and chunk offsets of the two-level scan (more than 2048
  // point blocks): kScanThreads block counts per chunk, records of 4 ints
  int *ctot, *ctot_b, *coff, *coff_b;
};
hipError_t launch_prep(const PrepCall& c);

// point blocks per chunk of the two-level offsets scan
constexpr int kScanThreads = 1024;
inline int64_t scan_chunks(int64_t nblk) { return (nblk + kScanThreads - 1) / kScanThreads; }

// Cut cells are walked by at most this many blocks of the residual launch
// (one loss partial each); the cell count itself is known only on the device.
constexpr int kCutBlocks = 1024;
inline int64_t cut_blocks(int64_t cut_cap) { return cut_cap < kCutBlocks ? cut_cap : kCutBlocks; }

struct ResCall {
  hipStream_t stream;
  Problem P;
  const Meta* meta;
  const float* pts;
  int64_t n;
  const float* bpts;
  int64_t nb;
  const int *cls, *rank, *bcls, *brank, *cutidx;
  int cut_cap;
  const float* outputs;
  float* adj;
  float* resid;
  double* lossp;
  double* loss;
  double scale;
  int skip_inline;
  int extra_parts;   // loss partials appended after the residual kernels' ones
  const float* fpre; // precomputed forcing per interior point, or NULL
  double* lacc;      // FP64 loss accumulator over resolution levels
  int acc;           // 0 one level; 1 first, 2 middle, 3 last of several
};
hipError_t launch_residuals(const ResCall& c);
hipError_t launch_reduce_loss(hipStream_t st, const double* lossp, int nparts, const Meta* meta,
                              double* loss);

hipError_t launch_fill(hipStream_t st, float* p, int64_t n, float v);
// Fourier forcing per interior point (f), and with fslot != NULL the same
// values in centre-slot order for uncut points
hipError_t launch_forcing(hipStream_t st, const Problem& P, const float* pts, int64_t n, float* f,
                          const Meta* meta, const int* cls, const int* rank, float* fslot);

// grad = scale * (FP64 fixed-order sum of the G partial rows); with `loss`,
// the same launch also reduces the nparts FP64 loss partials.  acc > 0
// accumulates resolution levels in the FP64 arrays gacc [P] and lacc [1].
hipError_t launch_reduce(hipStream_t st, const float* partial, int G, int64_t P, float* grad,
                         double scale, const double* lossp, int nparts, const Meta* meta, double* loss,
                         double* gacc, double* lacc, int acc);
hipError_t launch_adam(hipStream_t st, float* p, float* m, float* v, const float* g, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2);
hipError_t launch_sample_points(hipStream_t st, int dim, uint64_t seed, int64_t step, int64_t jh,
                                float* pts, int64_t n, float* bpts, int64_t nb);
hipError_t launch_counts(hipStream_t st, const Meta* meta, int* counts);
// multilinear interpolation of a nodal grid solution at one lattice tile
hipError_t launch_grid_interp(hipStream_t st, int dim, const double* U, int judge_n, int64_t tile_index,
                              int64_t m, int grid_n, float* u_out);
hipError_t launch_eval_out(hipStream_t st, int64_t slots, const Meta* meta, const float* outputs,
                           const int* src, float* u_out);

}  // namespace nbm
