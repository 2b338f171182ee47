// Internal types shared by the host launchers and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbm {

constexpr int kMaxDepth = 8;   // hidden layers supported
// threads per block of the Fourier forcing kernel; one phase row of its LDS
// table holds one float2 per thread, and the mode table's offsets are bytes
// into that table
constexpr int kForcingThreads = 128;
constexpr int kTile = 16;      // collocation centres per tile (MFMA M = 16)
constexpr int kBlock = 256;    // threads per work-group (4 wavefronts)

enum Kind { KIND_A = 0, KIND_B = 1, KIND_NBR = 2, KIND_BND = 3 };

// Problem description passed by value to kernels (paper Sec. 2).
// Fourier forcing modes for the per-point forcing kernel, grouped by
// (k_y, k_z), one record per mode, padded to a multiple of 8 with zero
// records.  Offsets address the per-thread phase table exp(i pi k x_a),
// k = 0..8, in LDS (entry a*9+k, rows of 256 threads x 8 bytes); negative
// wave numbers use the conjugate (bit 0 of oy/oz, sign folded into crs/cis).
struct FMode {
  int ox;                  // byte offset of the |k_x| phase row
  float cr, ci, crs, cis;  // c = a - i b, and c * sign(k_x)
  int oy, oz;              // the group's |k_y|, |k_z| rows; bit 0: negative
  int end;                 // 1 on the last mode of a (k_y, k_z) group
};

struct Problem {
  int dim, iface, kind, lo;   // lo: side with the smaller mu (0 minus, 1 plus), -1 if equal
  double R, amp, pn[3], pc;
  double mu[2];               // constant coefficients (mu_kind 0); with mu_kind 1 they only
                              // record which side has the smaller coefficient
  int mu_kind;                // 0 constant, 1 mu^- = y^2 ln(x+2) + 4, mu^+ = e^-z (Sec. 4.1)
  double kc[2];               // Helmholtz coefficients k^-+ of the term k u (>= 0)
  double alpha_c, beta_c;
  double lin_a[4], lin_b[4];
  double h;
  int n_modes;
  const float* modes32;   // [n_modes][8]: k0 k1 k2 a b - - -
  const double* modes64;  // [n_modes][5]: k0 k1 k2 a b
  int n_fmodes;           // padded count
  const FMode* fmodes;    // in group order
  int phi_n;              // level set on a coarse mesh: intervals per axis
  const double* phitab;   // its (phi_n + 1)^dim nodal values, axis 0 fastest
};

// Batch bookkeeping written on the device by the scan kernel.
struct Meta {
  int32_t cnt[2][4];   // centres per net and kind
  int32_t base[2][4];  // global slot of the first centre of (net, kind)
  int32_t total[2];    // centres per net
  int32_t tiles[2];    // tiles per net
  int32_t tile0[2];    // first global tile of each net
  int32_t ncls[3];     // interior points per class: A-, A+, cut
  int32_t nbside[2];   // boundary points per side
  int32_t nB;          // cut cells kept
  int32_t overflow;    // 1 if the cut capacity was exceeded
  int32_t n, nb;       // batch sizes
  int32_t slow;        // 1 if the 128-wide fast pass met an argument beyond its tier
};

// Per-net parameter pointers (FP32 master copy) and operand shadows.
struct NetPtrs {
  const float* W1;
  const float* b1;
  const float* bl[kMaxDepth];
  const float* wout;
  const float* bout;
  const void* Wl[kMaxDepth];    // shadow W_l [W][W] (operand dtype), l = 1..L-1 index = l-1
  const void* WlT[kMaxDepth];   // shadow W_l^T
  const float* Wf[kMaxDepth];   // FP32 master W_l (row-major), same index as Wl
};

struct Nets {
  NetPtrs net[2];
};

// Offsets (floats) of each parameter block inside one net.
struct NetLayout {
  int64_t W1, b1, Wl[kMaxDepth], bl[kMaxDepth], wout, bout, per_net;
};

}  // namespace nbm
