// C ABI of the NBM library (see include/nbm.h for the contract).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nbm.h"
#include "nbm_internal.hpp"
#include "nbm_launch.hpp"

using namespace nbm;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) return fail(NBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {
// Byte offsets of one call's workspace regions, for a batch of up to n
// interior and nb boundary points (or n queries).  The Fourier tables and the
// batch bookkeeping come first, at offsets that do not depend on the batch
// size (nbm_prepare fills the tables once; nbm_batch_counts reads the
// bookkeeping of the last call).
struct Layout {
  size_t modes32, modes64, fmodes, phitab, meta, prefix, ctot, coff, blockcnt, off, blockcnt_b, off_b, cls, rank, bcls,
      brank, cutidx, centres, src, outputs, adj, Zst, Ast, ALst, dZ, dZw, shadow, partial, lossp, resid, lossbuf,
      gacc, fpre, fslot, total;
  int64_t nchunk;    // interior chunks of the two-level scan
  int64_t cut_cap;   // cut cells this call can hold
  int64_t lstride;   // elements of one layer in the tile layout
};
}  // namespace

struct TimedPair {
  int group;
  hipEvent_t a, b;
};

struct nbm_ctx {
  bool timing = false;
  std::vector<TimedPair> timed;
  std::vector<hipEvent_t> pool;
  nbm_config cfg;
  std::vector<float> modes32;
  std::vector<double> modes64;
  std::vector<FMode> fmodes;
  std::vector<double> phitab;   // level-set mesh values (interface kind 3)
  Problem P;
  MlpFn mlp;
  EvalFn evalfn;   // persistent evaluation kernel, or null: the per-tile forward
  FusedFn fused;
  WideFn wide;
  int D, W, L, S, opbytes;
  int64_t per_net, Ptot;
  NetLayout lay;
  int64_t cap_n, cap_nb, cut_cap;   // largest batch (max_points, max_boundary) and cut capacity
  int G, Gf, Gfz;
  bool no_fused;
  Layout lo;        // layout at the largest batch (its prefix is shared by every call)
  void* prepared_ws;
  bool eval_only;
};

// event pair around one kernel group (no-op unless timing is enabled)
struct Timer {
  nbm_ctx* c;
  hipStream_t st;
  int group;
  hipEvent_t b_;
  bool on;
  Timer(nbm_ctx* c_, hipStream_t s, int g) : c(c_), st(s), group(g), b_(nullptr), on(c_->timing) {
    if (!on) return;
    hipEvent_t a;
    if (!c->pool.empty()) { a = c->pool.back(); c->pool.pop_back(); }
    else if (hipEventCreate(&a) != hipSuccess) { on = false; return; }
    if (!c->pool.empty()) { b_ = c->pool.back(); c->pool.pop_back(); }
    else if (hipEventCreate(&b_) != hipSuccess) { on = false; return; }
    (void)hipEventRecord(a, st);
    c->timed.push_back({group, a, b_});
  }
  ~Timer() {
    if (on) (void)hipEventRecord(b_, st);
  }
};

struct WideTimers {
  nbm_ctx* c;
  hipStream_t st;
  Timer* fb;
  Timer* dw;
};

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static Layout layout_for(const nbm_ctx* c, int64_t n, int64_t nb) {
  Layout L;
  size_t o = 0;
  const bool ev = c->eval_only;
  if (n < 1) n = 1;
  if (ev) nb = 0;
  // evaluation-only workspaces keep just the classification, centre lists,
  // outputs and operand shadows
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  auto take_tr = [&](size_t bytes) { return take(ev ? 0 : bytes); };
  const int64_t cut = ev ? 0 : std::min<int64_t>(c->cut_cap, n);
  const int nbr = c->P.lo >= 0 ? 2 * c->D : 0;
  const int64_t tiles = (n + (2 + nbr) * cut + nb + 2 * kTile + kTile - 1) / kTile + 2;
  const int64_t slots = tiles * kTile;
  L.cut_cap = cut;
  L.lstride = tiles * (int64_t)c->S * c->W * kTile;
  int64_t nblk = (n + 255) / 256 + 1, nblkb = (nb + 255) / 256 + 1;
  L.nchunk = scan_chunks(nblk);
  L.modes32 = take(sizeof(float) * 8 * (c->cfg.n_modes + 1));
  L.modes64 = take(sizeof(double) * 5 * (c->cfg.n_modes + 1));
  L.fmodes = take(sizeof(FMode) * (c->fmodes.size() + 1));
  L.phitab = take(sizeof(double) * (c->phitab.size() + 1));
  L.meta = take(sizeof(Meta));
  L.prefix = o;
  // chunk totals and offsets of the two-level scan: interior chunks, then
  // boundary chunks at a fixed offset
  L.ctot = take(sizeof(int) * 4 * (scan_chunks(nblk) + scan_chunks(nblkb)));
  L.coff = take(sizeof(int) * 4 * (scan_chunks(nblk) + scan_chunks(nblkb)));
  L.blockcnt = take(sizeof(int) * 4 * nblk);
  L.off = take(sizeof(int) * 4 * nblk);
  L.blockcnt_b = take(sizeof(int) * 4 * nblkb);
  L.off_b = take(sizeof(int) * 4 * nblkb);
  L.cls = take(sizeof(int) * n);
  L.rank = take(sizeof(int) * n);
  L.bcls = take(sizeof(int) * nb);
  L.brank = take(sizeof(int) * nb);
  L.cutidx = take(sizeof(int) * cut);
  L.centres = take(sizeof(float) * 4 * slots);
  L.src = take(sizeof(int) * slots);
  L.outputs = take(sizeof(float) * 8 * slots);
  L.adj = take_tr(sizeof(float) * 8 * slots);
  // stored pre-activations are needed only by the layered backward, used when
  // no fused path is compiled for the shape (or NBM_NO_FUSED is set)
  const bool layered = c->no_fused || (!c->fused && !c->wide);
  const bool two_pass = c->wide && !c->no_fused;
  L.Zst = take_tr(layered ? sizeof(float) * c->L * L.lstride : 0);
  // activations leave the chip only on the layered and the 128-wide two-pass paths
  L.Ast = take_tr(layered || two_pass ? (size_t)c->opbytes * (c->L - 1) * L.lstride : 0);
  L.ALst = take_tr(layered ? sizeof(float) * L.lstride : 0);
  L.dZ = take_tr(layered ? sizeof(float) * L.lstride : 0);
  L.dZw = take_tr(two_pass ? (size_t)c->opbytes * (c->L - 1) * L.lstride : 0);
  L.shadow = take((size_t)c->opbytes * 2 * (c->L - 1) * 2 * c->W * c->W);
  L.partial = take_tr(sizeof(float) * (size_t)c->G * c->Ptot);
  L.lossp = take(sizeof(double) * (nblk + nblkb + cut + 4 + 512));
  L.resid = take_tr(sizeof(float) * (n + nb));
  L.lossbuf = take(sizeof(double) * 4);
  // FP64 accumulators of the gradient and loss over resolution levels
  L.gacc = take_tr(c->cfg.levels > 0 ? sizeof(double) * (size_t)c->Ptot : 0);
  L.fpre = take_tr(c->cfg.problem == NBM_PROB_FOURIER ? sizeof(float) * n : 0);
  // forcing of the uncut centres in centre-slot order, for the fused paths'
  // inline tiles
  const bool fused_path = !c->no_fused && (c->fused || c->wide) && !c->eval_only;
  L.fslot = take_tr(fused_path ? sizeof(float) * slots : 0);
  L.total = o;
  return L;
}

extern "C" const char* nbm_last_error(void) { return g_err.c_str(); }

extern "C" int nbm_create(const nbm_config* cfg, nbm_ctx** out) {
  if (!cfg || !out) return fail(NBM_EINVAL, "null argument");
  const nbm_config& c = *cfg;
  if (c.dim != 2 && c.dim != 3) return fail(NBM_EINVAL, "dim must be 2 or 3");
  if (c.depth < 2 || c.depth > kMaxDepth) return fail(NBM_EINVAL, "depth must be in [2, 8]");
  if (c.act != NBM_ACT_TANH && c.act != NBM_ACT_SIN) return fail(NBM_EINVAL, "bad activation");
  if (c.prec != NBM_PREC_FP32 && c.prec != NBM_PREC_BF16) return fail(NBM_EINVAL, "bad precision");
  int h_exp = 0;
  if (!(c.h > 0.0) || c.h > 0.25 || c.h < std::ldexp(1.0, -20) || std::frexp(c.h, &h_exp) != 0.5)
    return fail(NBM_EINVAL, "h must be a power of two in [2^-20, 2^-2]");
  if (c.interface_kind < 0 || c.interface_kind > 3) return fail(NBM_EINVAL, "bad interface kind");
  if (c.interface_kind == NBM_IFACE_MESH) {
    if (c.phi_n < 2 || c.phi_n > 1024 || !c.phi_table)
      return fail(NBM_EINVAL, "the mesh level set needs phi_n in [2, 1024] and a table");
    const int64_t nv = (int64_t)std::pow((double)(c.phi_n + 1), c.dim);
    for (int64_t i = 0; i < nv; ++i)
      if (!std::isfinite(c.phi_table[i])) return fail(NBM_EINVAL, "level-set mesh values must be finite");
  }
  if (c.interface_kind == NBM_IFACE_STAR && c.dim != 3) return fail(NBM_EINVAL, "star needs dim 3");
  if (!(c.mu_minus > 0.0) || !(c.mu_plus > 0.0)) return fail(NBM_EINVAL, "mu must be positive");
  if (c.mu_kind < 0 || c.mu_kind > 1) return fail(NBM_EINVAL, "bad mu_kind");
  if (c.mu_kind == NBM_MU_PAPER && (c.dim != 3 || !(c.mu_plus < c.mu_minus)))
    return fail(NBM_EINVAL, "the Sec. 4.1 coefficients need dim 3 and mu_minus > mu_plus (mu^+ is the smaller side)");
  if (c.levels < 0 || c.levels > 6 || std::ldexp(c.h, -c.levels) < std::ldexp(1.0, -20))
    return fail(NBM_EINVAL, "levels must be in [0, 6] with h / 2^levels >= 2^-20");
  if (!(c.k_minus >= 0.0) || !(c.k_plus >= 0.0) || !std::isfinite(c.k_minus) || !std::isfinite(c.k_plus))
    return fail(NBM_EINVAL, "k must be finite and >= 0 (the discrete operator stays positive definite)");
  if (c.problem < 0 || c.problem > 3) return fail(NBM_EINVAL, "bad problem kind");
  if (c.problem == NBM_PROB_MMS_SPHERE && c.dim != 3) return fail(NBM_EINVAL, "problem needs dim 3");
  if (c.problem == NBM_PROB_FOURIER) {
    if (c.n_modes <= 0 || !c.mode_k || !c.mode_a || !c.mode_b)
      return fail(NBM_EINVAL, "Fourier problem needs a mode table");
    for (int m = 0; m < c.n_modes; ++m)
      for (int a = 0; a < 3; ++a)
        if (c.mode_k[3 * m + a] < -8 || c.mode_k[3 * m + a] > 8)
          return fail(NBM_EINVAL, "Fourier wave numbers must lie in [-8, 8]");
  }
  if (c.max_points < 1 || c.max_points > (1LL << 26) || c.max_boundary < 0 || c.max_boundary > (1LL << 24))
    return fail(NBM_EINVAL, "max_points must be in [1, 2^26], max_boundary in [0, 2^24]");
  if (!c.eval_only && c.max_points > (1LL << 24))
    return fail(NBM_EINVAL, "training batches are limited to 2^24 points (use eval_only for larger tiles)");
  MlpFn fn = find_mlp(c.dim, c.width, c.act, c.prec);
  if (!fn)
    return fail(NBM_EUNSUPPORTED, "no kernel compiled for (dim, width, act, prec) = (" +
                                      std::to_string(c.dim) + ", " + std::to_string(c.width) + ", " +
                                      std::to_string(c.act) + ", " + std::to_string(c.prec) + ")");
  nbm_ctx* x = new (std::nothrow) nbm_ctx();
  if (!x) return fail(NBM_EINVAL, "out of host memory");
  x->cfg = c;
  x->cfg.mode_k = nullptr;
  x->cfg.mode_a = x->cfg.mode_b = nullptr;
  x->cfg.phi_table = nullptr;
  if (c.interface_kind == NBM_IFACE_MESH)
    x->phitab.assign(c.phi_table, c.phi_table + (size_t)std::pow((double)(c.phi_n + 1), c.dim));
  x->mlp = fn;
  x->evalfn = find_eval(c.dim, c.width, c.depth, c.act, c.prec);
  x->fused = find_fused(c.dim, c.width, c.depth, c.act, c.prec);
  x->wide = find_wide(c.dim, c.width, c.depth, c.act, c.prec);
  // the fused kernels form the uncut residual of constant coefficients in
  // their epilogue; variable coefficients take the layered path, whose
  // residual kernel weights each face by mu at its centre
  x->no_fused = std::getenv("NBM_NO_FUSED") != nullptr || c.mu_kind != NBM_MU_CONST;
  x->D = c.dim; x->W = c.width; x->L = c.depth; x->S = 2 * c.dim + 1;
  x->opbytes = c.prec == NBM_PREC_BF16 ? 2 : 4;
  // parameter layout of one net
  NetLayout& ly = x->lay;
  int64_t o = 0, W = c.width, D = c.dim;
  ly.W1 = o; o += W * D;
  ly.b1 = o; o += W;
  for (int l = 0; l < kMaxDepth; ++l) { ly.Wl[l] = 0; ly.bl[l] = 0; }
  for (int l = 0; l < c.depth - 1; ++l) { ly.Wl[l] = o; o += W * W; ly.bl[l] = o; o += W; }
  ly.wout = o; o += W;
  ly.bout = o; o += 1;
  ly.per_net = o;
  x->per_net = o;
  x->Ptot = 2 * o;
  // problem
  Problem& P = x->P;
  std::memset(&P, 0, sizeof(P));
  P.dim = c.dim; P.iface = c.interface_kind; P.kind = c.problem;
  P.R = c.radius; P.amp = c.star_amp;
  for (int a = 0; a < 3; ++a) P.pn[a] = c.plane_n[a];
  P.pc = c.plane_c;
  P.mu[0] = c.mu_minus; P.mu[1] = c.mu_plus;
  P.mu_kind = c.mu_kind;
  P.kc[0] = c.k_minus; P.kc[1] = c.k_plus;
  P.lo = c.mu_minus == c.mu_plus ? -1 : (c.mu_minus < c.mu_plus ? 0 : 1);
  P.alpha_c = c.alpha_const; P.beta_c = c.beta_const;
  for (int a = 0; a < 4; ++a) { P.lin_a[a] = c.lin_a[a]; P.lin_b[a] = c.lin_b[a]; }
  P.h = c.h;
  P.phi_n = c.interface_kind == NBM_IFACE_MESH ? c.phi_n : 0;
  P.n_modes = c.problem == NBM_PROB_FOURIER ? c.n_modes : 0;
  if (P.n_modes) {
    x->modes32.assign(8 * (size_t)P.n_modes, 0.0f);
    x->modes64.assign(5 * (size_t)P.n_modes, 0.0);
    for (int m = 0; m < P.n_modes; ++m) {
      for (int a = 0; a < 3; ++a) {
        x->modes32[8 * m + a] = (float)c.mode_k[3 * m + a];
        x->modes64[5 * m + a] = (double)c.mode_k[3 * m + a];
      }
      x->modes32[8 * m + 3] = (float)c.mode_a[m];
      x->modes32[8 * m + 4] = (float)c.mode_b[m];
      x->modes64[5 * m + 3] = c.mode_a[m];
      x->modes64[5 * m + 4] = c.mode_b[m];
    }
    // grouped by (k_y, k_z): a*cos(pi k.x) + b*sin(pi k.x) = Re(c e^{i pi k.x}),
    // c = a - i b; e^{-i t} = conj(e^{i t}) handles negative wave numbers
    std::map<std::pair<int, int>, std::vector<int>> byyz;
    for (int m = 0; m < P.n_modes; ++m) byyz[{c.mode_k[3 * m + 1], c.mode_k[3 * m + 2]}].push_back(m);
    constexpr int kRow = kForcingThreads * 8;   // bytes per phase row (one float2 per thread)
    // the forcing kernel's phase rows: 0 holds 1 (k = 0 on any axis), 1..8
    // k_x = 1..8, 9..12 k_y = 1..4, 13..16 k_z = 1..4; a y or z offset with
    // bit 1 set names the row of |k| - 4, to be multiplied by that of 4;
    // bit 0 marks a negative wave number
    auto yz_off = [](int a, int k) {
      const int m = std::abs(k), r = m == 0 ? 0 : 4 * a + 4 + (m > 4 ? m - 4 : m);
      return r * kRow + (m > 4 ? 2 : 0) + (k < 0 ? 1 : 0);
    };
    for (const auto& kv : byyz) {
      const int ky = kv.first.first, kz = kv.first.second;
      const int oy = yz_off(1, ky);
      const int oz = yz_off(2, kz);
      for (size_t q = 0; q < kv.second.size(); ++q) {
        const int m = kv.second[q];
        FMode M;
        std::memset(&M, 0, sizeof(M));
        const int kx = c.mode_k[3 * m];
        const float sx = kx < 0 ? -1.0f : 1.0f;
        M.ox = std::abs(kx) * kRow;
        M.cr = (float)c.mode_a[m];
        M.ci = (float)(-c.mode_b[m]);
        M.crs = M.cr * sx;
        M.cis = M.ci * sx;
        M.oy = oy;
        M.oz = oz;
        M.end = q + 1 == kv.second.size() ? 1 : 0;
        x->fmodes.push_back(M);
      }
    }
    while (x->fmodes.size() % 8) {
      FMode Z;
      std::memset(&Z, 0, sizeof(Z));
      x->fmodes.push_back(Z);
    }
    P.n_fmodes = (int)x->fmodes.size();
  }
  x->cfg.n_modes = P.n_modes;
  // capacities
  x->eval_only = c.eval_only != 0;
  x->cap_n = c.max_points;
  x->cap_nb = c.max_boundary;
  x->cut_cap = c.cut_capacity > 0 ? c.cut_capacity : c.max_points / 8 + 64;
  if (x->cut_cap > x->cap_n) x->cut_cap = x->cap_n;
  if (x->eval_only) { x->cut_cap = 0; x->cap_nb = 0; }
  x->G = 512;
  x->Gf = 256;
  x->Gfz = 512;   // two fused work-groups per compute unit
  x->prepared_ws = nullptr;
  x->lo = layout_for(x, x->cap_n, x->cap_nb);
  *out = x;
  return NBM_OK;
}

extern "C" void nbm_destroy(nbm_ctx* ctx) {
  if (!ctx) return;
  for (auto& t : ctx->timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  for (auto& e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
}

extern "C" int nbm_set_timing(nbm_ctx* ctx, int enable) {
  if (!ctx) return fail(NBM_EINVAL, "null context");
  ctx->timing = enable != 0;
  return NBM_OK;
}

extern "C" int nbm_read_timing(nbm_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx || !ms || !launches) return fail(NBM_EINVAL, "null argument");
  for (int g = 0; g < NBM_TIMING_GROUPS; ++g) { ms[g] = 0.0; launches[g] = 0; }
  for (auto& t : ctx->timed) {
    HIPCHK(hipEventSynchronize(t.b));
    float v = 0.f;
    HIPCHK(hipEventElapsedTime(&v, t.a, t.b));
    ms[t.group] += v;
    launches[t.group] += 1;
    ctx->pool.push_back(t.a);
    ctx->pool.push_back(t.b);
  }
  ctx->timed.clear();
  return NBM_OK;
}

extern "C" int64_t nbm_param_count(const nbm_ctx* ctx) { return ctx ? ctx->Ptot : -1; }

extern "C" size_t nbm_workspace_bytes(const nbm_ctx* ctx, int64_t n, int64_t nb) {
  if (!ctx || n < 0 || nb < 0 || n > ctx->cap_n || nb > ctx->cap_nb) return 0;
  return layout_for(ctx, n, nb).total;
}

template <class T>
static T* at(void* ws, size_t off) {
  return (T*)((char*)ws + off);
}

static int check_ws(nbm_ctx* ctx, void* ws, size_t bytes, const Layout& need) {
  if (!ws) return fail(NBM_EWORKSPACE, "workspace is null");
  if (bytes < need.total) return fail(NBM_EWORKSPACE, "workspace too small: need " + std::to_string(need.total));
  if (ctx->prepared_ws != ws) return fail(NBM_EWORKSPACE, "workspace not prepared (call nbm_prepare)");
  if (((uintptr_t)ws & 255) != 0) return fail(NBM_EWORKSPACE, "workspace must be 256-byte aligned");
  return NBM_OK;
}

extern "C" int nbm_prepare(nbm_ctx* ctx, void* stream, void* ws, size_t ws_bytes) {
  if (!ctx || !ws) return fail(NBM_EINVAL, "null argument");
  if (ws_bytes < ctx->lo.prefix) return fail(NBM_EWORKSPACE, "workspace too small: need " + std::to_string(ctx->lo.prefix));
  if (((uintptr_t)ws & 255) != 0) return fail(NBM_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  if (!ctx->phitab.empty()) {
    HIPCHK(hipMemcpyAsync(at<char>(ws, ctx->lo.phitab), ctx->phitab.data(), sizeof(double) * ctx->phitab.size(),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (ctx->P.n_modes) {
    HIPCHK(hipMemcpyAsync(at<char>(ws, ctx->lo.modes32), ctx->modes32.data(), sizeof(float) * ctx->modes32.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at<char>(ws, ctx->lo.modes64), ctx->modes64.data(), sizeof(double) * ctx->modes64.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at<char>(ws, ctx->lo.fmodes), ctx->fmodes.data(), sizeof(FMode) * ctx->fmodes.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  ctx->prepared_ws = ws;
  return NBM_OK;
}

static Problem problem_for(nbm_ctx* ctx, void* ws) {
  Problem P = ctx->P;
  P.modes32 = at<float>(ws, ctx->lo.modes32);
  P.modes64 = at<double>(ws, ctx->lo.modes64);
  P.fmodes = at<FMode>(ws, ctx->lo.fmodes);
  P.phitab = at<double>(ws, ctx->lo.phitab);
  return P;
}

static Nets nets_for(nbm_ctx* ctx, const float* params, void* ws, const Layout& Lo) {
  Nets N;
  std::memset(&N, 0, sizeof(N));
  size_t wsz = (size_t)ctx->W * ctx->W * ctx->opbytes;
  char* sh = at<char>(ws, Lo.shadow);
  for (int net = 0; net < 2; ++net) {
    const float* p = params + net * ctx->per_net;
    NetPtrs& np = N.net[net];
    np.W1 = p + ctx->lay.W1;
    np.b1 = p + ctx->lay.b1;
    np.wout = p + ctx->lay.wout;
    np.bout = p + ctx->lay.bout;
    for (int l = 0; l < ctx->L - 1; ++l) {
      np.bl[l] = p + ctx->lay.bl[l];
      np.Wf[l] = p + ctx->lay.Wl[l];
      np.Wl[l] = sh + ((size_t)(net * (ctx->L - 1) + l) * 2 + 0) * wsz;
      np.WlT[l] = sh + ((size_t)(net * (ctx->L - 1) + l) * 2 + 1) * wsz;
    }
  }
  return N;
}

static int check_points(nbm_ctx* ctx, const float* pts, int64_t n, const float* bpts, int64_t nb) {
  if (ctx->eval_only) return fail(NBM_EWORKSPACE, "context was created with eval_only");
  if (n < 0 || nb < 0) return fail(NBM_EINVAL, "negative batch size");
  if (n + nb == 0) return fail(NBM_EINVAL, "empty batch");
  if (n > ctx->cap_n || nb > ctx->cap_nb) return fail(NBM_EINVAL, "batch exceeds max_points / max_boundary");
  if (n > 0 && !pts) return fail(NBM_EINVAL, "pts is null");
  if (nb > 0 && !bpts) return fail(NBM_EINVAL, "bpts is null");
  return NBM_OK;
}

// the hidden matrices of both networks, for one operand-copy launch
static ShadowJobs shadow_jobs(const nbm_ctx* ctx, const float* params, const Nets& N) {
  ShadowJobs j;
  std::memset(&j, 0, sizeof(j));
  j.params = params;
  j.W = ctx->W;
  for (int net = 0; net < 2; ++net)
    for (int l = 0; l < ctx->L - 1; ++l) {
      j.off[j.count] = net * ctx->per_net + ctx->lay.Wl[l];
      j.Wl[j.count] = (void*)N.net[net].Wl[l];
      j.WlT[j.count] = (void*)N.net[net].WlT[l];
      ++j.count;
    }
  return j;
}

// forward (+ optional backward) of one batch at one resolution: implicit
// cells of side h; acc says how the level's loss and gradient enter the
// FP64 accumulators (0: a single level)
static int run_level(nbm_ctx* ctx, hipStream_t st, const float* params, const float* pts, int64_t n,
                     const float* bpts, int64_t nb, float* residual, double* loss, float* grad,
                     double dL, void* ws, const Layout& Lo, double h, int acc) {
  Problem P = problem_for(ctx, ws);
  P.h = h;
  double* gacc = at<double>(ws, Lo.gacc);
  double* lacc = at<double>(ws, Lo.lossbuf) + 1;
  // operand shadows of the hidden matrices
  Nets N = nets_for(ctx, params, ws, Lo);
  Timer* tprep = new Timer(ctx, st, 0);

  // classification and centre lists
  PrepCall pc;
  std::memset(&pc, 0, sizeof(pc));
  pc.stream = st; pc.P = P; pc.pts = pts; pc.n = n; pc.bpts = bpts; pc.nb = nb; pc.eval = false;
  pc.cut_cap = (int)Lo.cut_cap;
  pc.cls = at<int>(ws, Lo.cls); pc.rank = at<int>(ws, Lo.rank);
  pc.blockcnt = at<int>(ws, Lo.blockcnt); pc.off = at<int>(ws, Lo.off);
  pc.bcls = at<int>(ws, Lo.bcls); pc.brank = at<int>(ws, Lo.brank);
  pc.blockcnt_b = at<int>(ws, Lo.blockcnt_b); pc.off_b = at<int>(ws, Lo.off_b);
  pc.meta = at<Meta>(ws, Lo.meta);
  pc.ctot = at<int>(ws, Lo.ctot); pc.ctot_b = pc.ctot + 4 * Lo.nchunk;
  pc.coff = at<int>(ws, Lo.coff); pc.coff_b = pc.coff + 4 * Lo.nchunk;
  pc.centres = at<float4>(ws, Lo.centres);
  pc.src = at<int>(ws, Lo.src);
  pc.cutidx = at<int>(ws, Lo.cutidx);
  pc.shadows = shadow_jobs(ctx, params, N);
  pc.prec = ctx->cfg.prec;
  // the fused kernels read the forcing of their uncut centres in slot order:
  // the manufactured forcing is written by the scatter, the Fourier forcing
  // by its own kernel
  const bool fused_step = grad != nullptr && (ctx->fused != nullptr || ctx->wide != nullptr) && !ctx->no_fused;
  float* f_inline = fused_step ? at<float>(ws, Lo.fslot) : nullptr;
  const bool fourier = ctx->cfg.problem == NBM_PROB_FOURIER;
  pc.fslot = fourier ? nullptr : f_inline;
  hipError_t e = launch_prep(pc);
  delete tprep;
  const float* fpre = nullptr;
  if (fourier && n > 0) {
    fpre = at<float>(ws, Lo.fpre);
    Timer tfo(ctx, st, 9);
    if (e == hipSuccess) e = launch_forcing(st, P, pts, n, (float*)fpre, pc.meta, pc.cls, pc.rank, f_inline);
  }
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("prep: ") + hipGetErrorString(e));
  // network streams at every centre
  int nbr = P.lo >= 0 ? 2 * ctx->D : 0;
  const int64_t cut_here = Lo.cut_cap;
  int64_t slots = n + (2 + nbr) * cut_here + nb + 2 * kTile;
  int grid = (int)((slots + kTile - 1) / kTile + 2);
  const bool fused = grad != nullptr && (ctx->fused != nullptr || ctx->wide != nullptr) && !ctx->no_fused;
  MlpCall mc;
  std::memset(&mc, 0, sizeof(mc));
  mc.op = MlpCall::FORWARD; mc.stream = st; mc.grid = grid; mc.meta = pc.meta;
  mc.centres = pc.centres; mc.nets = &N; mc.L = ctx->L; mc.h = (float)h;
  mc.outputs = at<float>(ws, Lo.outputs);
  mc.Zst = at<float>(ws, Lo.Zst); mc.Ast = at<void>(ws, Lo.Ast); mc.ALst = at<float>(ws, Lo.ALst);
  mc.dZ = at<float>(ws, Lo.dZ); mc.lstride = Lo.lstride;
  mc.store = grad != nullptr && !fused; mc.streams = true;
  if (fused) {
    // forward only over the tiles that are not 16 uncut centres
    mc.noninline = 1;
    // the kernel walks the tiles with the grid as stride (their number is
    // known only on the device): two resident blocks per compute unit
    mc.grid = (int)std::min<int64_t>(((2 + nbr) * cut_here + nb + kTile - 1) / kTile + 6, 512);
  }
  {
    Timer tf(ctx, st, 1);
    e = ctx->mlp(mc);
  }
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("forward: ") + hipGetErrorString(e));
  // residuals, loss and output adjoints
  float* adj = at<float>(ws, Lo.adj);
  Timer* tres = new Timer(ctx, st, 2);
  if (grad && !fused) {
    // the layered backward reads every slot's adjoints (the fused kernels only
    // those the residual kernels write in full)
    e = launch_fill(st, adj, (int64_t)grid * kTile * 8, 0.0f);
    if (e != hipSuccess) { delete tres; return fail(NBM_EHIP, std::string("fill: ") + hipGetErrorString(e)); }
  }
  ResCall rc;
  std::memset(&rc, 0, sizeof(rc));
  rc.stream = st; rc.P = P; rc.meta = pc.meta; rc.pts = pts; rc.n = n; rc.bpts = bpts; rc.nb = nb;
  rc.cls = pc.cls; rc.rank = pc.rank; rc.bcls = pc.bcls; rc.brank = pc.brank; rc.cutidx = pc.cutidx;
  rc.cut_cap = (int)cut_here;
  rc.outputs = mc.outputs; rc.adj = adj;
  rc.resid = residual ? residual : at<float>(ws, Lo.resid);
  rc.lossp = at<double>(ws, Lo.lossp);
  double* loss_out = loss ? loss : at<double>(ws, Lo.lossbuf);
  rc.loss = fused ? nullptr : loss_out;
  rc.scale = 2.0 * dL / (double)(n + nb);
  rc.skip_inline = fused ? 1 : 0;
  rc.fpre = fpre;
  rc.lacc = lacc;
  rc.acc = acc;
  e = launch_residuals(rc);
  delete tres;
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("residual: ") + hipGetErrorString(e));
  if (!grad) return NBM_OK;
  float* partial = at<float>(ws, Lo.partial);
  int Grows = ctx->G;
  // the fused paths' loss partials are reduced in the gradient reduction's launch
  const double* red_lossp = nullptr;
  int red_nparts = 0;
  double* red_loss = nullptr;
  if (fused && ctx->wide) {
    int nres = (int)((n + 255) / 256 + (n ? cut_blocks(cut_here) : 0) + (nb + 255) / 256);
    WideCall wc;
    std::memset(&wc, 0, sizeof(wc));
    wc.stream = st; wc.grid = ctx->Gf; wc.meta = pc.meta; wc.centres = pc.centres; wc.src = pc.src;
    wc.nets = &N; wc.P = P; wc.h = (float)h; wc.adj = adj; wc.resid = rc.resid;
    wc.A = at<void>(ws, Lo.Ast); wc.dZ = at<void>(ws, Lo.dZw); wc.lstride = Lo.lstride;
    wc.partial = partial; wc.Ptot = ctx->Ptot; wc.lay = &ctx->lay; wc.off1 = ctx->per_net;
    wc.lossp = rc.lossp + nres; wc.scale = rc.scale; wc.fslot = f_inline;
    // group 3 times the forward/backward launch, group 8 each weight-gradient launch
    WideTimers wt{ctx, st, new Timer(ctx, st, 3), nullptr};
    wc.timer_ctx = &wt;
    wc.after_fb = [](void* p) { auto* t = (WideTimers*)p; delete t->fb; t->fb = nullptr; };
    wc.timer_begin = [](void* p) { auto* t = (WideTimers*)p; t->dw = new Timer(t->c, t->st, 8); };
    wc.timer_end = [](void* p) { auto* t = (WideTimers*)p; delete t->dw; t->dw = nullptr; };
    e = ctx->wide(wc);
    delete wt.fb;
    delete wt.dw;
    if (e != hipSuccess) return fail(NBM_EHIP, std::string("wide: ") + hipGetErrorString(e));
    red_lossp = rc.lossp; red_nparts = nres + ctx->Gf; red_loss = loss_out;
    Grows = ctx->Gf;
  } else if (fused) {
    int nres = (int)((n + 255) / 256 + (n ? cut_blocks(cut_here) : 0) + (nb + 255) / 256);
    FusedCall fc;
    std::memset(&fc, 0, sizeof(fc));
    fc.stream = st; fc.grid = ctx->Gfz; fc.meta = pc.meta; fc.centres = pc.centres; fc.src = pc.src;
    fc.nets = &N; fc.P = P; fc.h = (float)h; fc.adj = adj; fc.resid = rc.resid;
    fc.partial = partial; fc.Ptot = ctx->Ptot; fc.lay = &ctx->lay; fc.off1 = ctx->per_net;
    fc.lossp = rc.lossp + nres; fc.scale = rc.scale; fc.fslot = f_inline;
    {
      Timer tb(ctx, st, 3);
      e = ctx->fused(fc);
    }
    if (e != hipSuccess) return fail(NBM_EHIP, std::string("fused: ") + hipGetErrorString(e));
    red_lossp = rc.lossp; red_nparts = nres + ctx->Gfz; red_loss = loss_out;
    Grows = ctx->Gfz;
  } else {
    // backward through the hidden layers, gradient partials
    mc.op = MlpCall::BACKWARD;
    mc.grid = ctx->G;
    mc.adj = adj;
    mc.partial = partial;
    mc.Ptot = ctx->Ptot;
    mc.lay = &ctx->lay;
    mc.off1 = ctx->per_net;
    for (int l = ctx->L; l >= 2; --l) {
      mc.l = l;
      {
        Timer tb(ctx, st, 3);
        e = ctx->mlp(mc);
      }
      if (e != hipSuccess) return fail(NBM_EHIP, std::string("backward: ") + hipGetErrorString(e));
    }
  }
  {
    Timer tr(ctx, st, 4);
    e = launch_reduce(st, partial, Grows, ctx->Ptot, grad, 1.0, red_lossp, red_nparts, pc.meta, red_loss, gacc,
                      lacc, acc);
  }
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("reduce: ") + hipGetErrorString(e));
  return NBM_OK;
}

// One batch over every resolution level (paper Sec. 3: implicit cells of
// several resolutions at each collocation point; Sec. 4.2: a base
// resolution refined implicitly): level l uses cells of side h / 2^l and
// the levels' losses and gradients are summed in FP64.
static int run_step(nbm_ctx* ctx, hipStream_t st, const float* params, const float* pts, int64_t n,
                    const float* bpts, int64_t nb, float* residual, double* loss, float* grad,
                    double dL, void* ws, const Layout& Lo) {
  const int R = ctx->cfg.levels;
  for (int l = 0; l <= R; ++l) {
    const int acc = R == 0 ? 0 : (l == 0 ? 1 : (l == R ? 3 : 2));
    float* res_l = residual ? residual + (int64_t)l * (n + nb) : nullptr;
    const int rc = run_level(ctx, st, params, pts, n, bpts, nb, res_l, loss, grad, dL, ws, Lo,
                             std::ldexp(ctx->cfg.h, -l), acc);
    if (rc) return rc;
  }
  return NBM_OK;
}

extern "C" int nbm_forward_residual(nbm_ctx* ctx, void* stream, const float* params, const float* pts,
                                    int64_t n, const float* bpts, int64_t nb, float* residual,
                                    double* loss, float* grad, void* ws, size_t ws_bytes) {
  if (!ctx || !params || !loss) return fail(NBM_EINVAL, "null argument");
  int rc = check_points(ctx, pts, n, bpts, nb);
  if (rc) return rc;
  const Layout Lo = layout_for(ctx, n, nb);
  rc = check_ws(ctx, ws, ws_bytes, Lo);
  if (rc) return rc;
  return run_step(ctx, (hipStream_t)stream, params, pts, n, bpts, nb, residual, loss, grad, 1.0, ws, Lo);
}

extern "C" int nbm_backward(nbm_ctx* ctx, void* stream, const float* params, const float* pts, int64_t n,
                            const float* bpts, int64_t nb, double dL, float* grad, void* ws,
                            size_t ws_bytes) {
  if (!ctx || !params || !grad) return fail(NBM_EINVAL, "null argument");
  if (!std::isfinite(dL)) return fail(NBM_EINVAL, "dL must be finite");
  int rc = check_points(ctx, pts, n, bpts, nb);
  if (rc) return rc;
  const Layout Lo = layout_for(ctx, n, nb);
  rc = check_ws(ctx, ws, ws_bytes, Lo);
  if (rc) return rc;
  return run_step(ctx, (hipStream_t)stream, params, pts, n, bpts, nb, nullptr, nullptr, grad, dL, ws, Lo);
}

// Scratch of the allocation-free entry point: one copy of this array per GPU,
// held until the process ends.  Host code never uses the array's name as an
// address: the device address of this GPU's copy comes from
// hipGetSymbolAddress, once per device, with that device current.
static_assert(NBM_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of 256 bytes");
static __device__ __align__(256) unsigned char scratch[NBM_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices];

static int scratch_of_current_device(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NBM_EHIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(NBM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return NBM_OK;
}

extern "C" int nbm_forward_residual_noalloc(nbm_ctx* ctx, void* stream, const float* params,
                                            const float* pts, int64_t n, const float* bpts, int64_t nb,
                                            float* residual, double* loss, float* grad) {
  if (!ctx || !params || !loss) return fail(NBM_EINVAL, "null argument");
  if (ctx->P.n_modes)
    return fail(NBM_EUNSUPPORTED, "the allocation-free entry point does not serve the Fourier problem "
                                  "(its mode tables would need a host-to-device copy): use "
                                  "nbm_forward_residual with a prepared workspace");
  int rc = check_points(ctx, pts, n, bpts, nb);
  if (rc) return rc;
  const Layout Lo = layout_for(ctx, n, nb);
  if (Lo.total > (size_t)NBM_SCRATCH_BYTES)
    return fail(NBM_EWORKSPACE, "batch needs " + std::to_string(Lo.total) + " bytes of scratch; the "
                                "allocation-free entry point holds " + std::to_string((size_t)NBM_SCRATCH_BYTES) +
                                " (use nbm_forward_residual with a workspace)");
  void* ws = nullptr;
  rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  // every region the step reads is written earlier in the same call (the
  // batch bookkeeping by the scan, partial rows and loss partials by their
  // kernels), so nothing needs clearing between calls
  return run_step(ctx, (hipStream_t)stream, params, pts, n, bpts, nb, residual, loss, grad, 1.0, ws, Lo);
}

extern "C" int nbm_adam_step(nbm_ctx* ctx, void* stream, float* params, float* m, float* v,
                             const float* grad, int64_t step, float lr, float beta1, float beta2,
                             float eps) {
  if (!ctx || !params || !m || !v || !grad) return fail(NBM_EINVAL, "null argument");
  if (step < 1) return fail(NBM_EINVAL, "step is 1-based");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return fail(NBM_EINVAL, "bad Adam hyper-parameters");
  double c1 = 1.0 - std::pow((double)beta1, (double)step), c2 = 1.0 - std::pow((double)beta2, (double)step);
  Timer ta(ctx, (hipStream_t)stream, 5);
  hipError_t e = launch_adam((hipStream_t)stream, params, m, v, grad, ctx->Ptot, lr, beta1, beta2, eps,
                             (float)c1, (float)c2);
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("adam: ") + hipGetErrorString(e));
  return NBM_OK;
}

extern "C" int nbm_sample_points(nbm_ctx* ctx, void* stream, uint64_t seed, int64_t step, float* pts,
                                 int64_t n, float* bpts, int64_t nb) {
  if (!ctx) return fail(NBM_EINVAL, "null context");
  if (n < 0 || nb < 0 || (n && !pts) || (nb && !bpts)) return fail(NBM_EINVAL, "bad point buffers");
  if (step < 0) return fail(NBM_EINVAL, "negative step");
  int64_t jh = (int64_t)std::llround(ctx->cfg.h * (double)(1 << 22));
  Timer ts(ctx, (hipStream_t)stream, 6);
  hipError_t e = launch_sample_points((hipStream_t)stream, ctx->D, seed, step, jh, pts, n, bpts, nb);
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("sample: ") + hipGetErrorString(e));
  return NBM_OK;
}

extern "C" int nbm_eval(nbm_ctx* ctx, void* stream, const float* params, const float* query, int64_t m,
                        int64_t tile_index, int32_t grid_n, float* u_out, void* ws, size_t ws_bytes) {
  if (!ctx || !params || !u_out) return fail(NBM_EINVAL, "null argument");
  if (m < 1 || m > ctx->cap_n) return fail(NBM_EINVAL, "m must be in [1, max_points]");
  const Layout Lo = layout_for(ctx, m, 0);
  int rc = check_ws(ctx, ws, ws_bytes, Lo);
  if (rc) return rc;
  if (!query) {
    if (grid_n < 2 || (grid_n & (grid_n - 1)) != 0 || grid_n > (1 << 14))
      return fail(NBM_EINVAL, "grid_n must be a power of two in [2, 2^14]");
    double tot = std::pow((double)grid_n, ctx->D);
    if (tile_index < 0 || (double)(tile_index + 1) * (double)m > tot)
      return fail(NBM_EINVAL, "tile outside the grid");
  }
  hipStream_t st = (hipStream_t)stream;
  Problem P = problem_for(ctx, ws);
  Nets N = nets_for(ctx, params, ws, Lo);
  Timer tev(ctx, st, 7);

  PrepCall pc;
  std::memset(&pc, 0, sizeof(pc));
  pc.stream = st; pc.P = P; pc.pts = query; pc.n = m; pc.bpts = nullptr; pc.nb = 0; pc.eval = true;
  pc.tile_index = tile_index; pc.grid_n = grid_n;
  pc.cut_cap = 0;
  pc.cls = at<int>(ws, Lo.cls); pc.rank = at<int>(ws, Lo.rank);
  pc.blockcnt = at<int>(ws, Lo.blockcnt); pc.off = at<int>(ws, Lo.off);
  pc.bcls = at<int>(ws, Lo.bcls); pc.brank = at<int>(ws, Lo.brank);
  pc.blockcnt_b = at<int>(ws, Lo.blockcnt_b); pc.off_b = at<int>(ws, Lo.off_b);
  pc.meta = at<Meta>(ws, Lo.meta);
  pc.ctot = at<int>(ws, Lo.ctot); pc.ctot_b = pc.ctot + 4 * Lo.nchunk;
  pc.coff = at<int>(ws, Lo.coff); pc.coff_b = pc.coff + 4 * Lo.nchunk;
  pc.centres = at<float4>(ws, Lo.centres);
  pc.src = at<int>(ws, Lo.src);
  pc.cutidx = at<int>(ws, Lo.cutidx);
  pc.shadows = shadow_jobs(ctx, params, N);
  pc.prec = ctx->cfg.prec;
  hipError_t e = launch_prep(pc);
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("prep: ") + hipGetErrorString(e));
  if (ctx->evalfn) {
    EvalCall ec;
    std::memset(&ec, 0, sizeof(ec));
    ec.stream = st;
    ec.max_grid = (int)std::min<int64_t>((m + 63) / 64 + 2, 1 << 20);   // tiles of 64 centres, both nets
    ec.meta = pc.meta; ec.centres = pc.centres; ec.src = pc.src; ec.nets = &N; ec.u_out = u_out;
    e = ctx->evalfn(ec);
    if (e != hipSuccess) return fail(NBM_EHIP, std::string("eval: ") + hipGetErrorString(e));
    return NBM_OK;
  }
  int64_t slots = m + 2 * kTile;
  int grid = (int)((slots + kTile - 1) / kTile + 2);
  MlpCall mc;
  std::memset(&mc, 0, sizeof(mc));
  mc.op = MlpCall::FORWARD; mc.stream = st; mc.grid = grid; mc.meta = pc.meta;
  mc.centres = pc.centres; mc.nets = &N; mc.L = ctx->L; mc.h = (float)ctx->cfg.h;
  mc.outputs = at<float>(ws, Lo.outputs);
  mc.lstride = Lo.lstride;
  mc.store = false; mc.streams = false;
  e = ctx->mlp(mc);
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("eval: ") + hipGetErrorString(e));
  e = launch_eval_out(st, (int64_t)grid * kTile, pc.meta, mc.outputs, pc.src, u_out);
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("eval out: ") + hipGetErrorString(e));
  return NBM_OK;
}

extern "C" int nbm_grid_interp(nbm_ctx* ctx, void* stream, const double* U, int32_t judge_n,
                               int64_t tile_index, int32_t grid_n, int64_t m, float* u_out) {
  if (!ctx || !U || !u_out) return fail(NBM_EINVAL, "null argument");
  if (judge_n < 1 || judge_n > (1 << 14)) return fail(NBM_EINVAL, "judge_n must be in [1, 2^14]");
  if (grid_n < 2 || (grid_n & (grid_n - 1)) != 0 || grid_n > (1 << 14))
    return fail(NBM_EINVAL, "grid_n must be a power of two in [2, 2^14]");
  if (m < 1) return fail(NBM_EINVAL, "m must be positive");
  const double tot = std::pow((double)grid_n, ctx->D);
  if (tile_index < 0 || (double)(tile_index + 1) * (double)m > tot)
    return fail(NBM_EINVAL, "tile outside the grid");
  Timer tev(ctx, (hipStream_t)stream, 7);
  hipError_t e = launch_grid_interp((hipStream_t)stream, ctx->D, U, judge_n, tile_index, m, grid_n, u_out);
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("grid interp: ") + hipGetErrorString(e));
  return NBM_OK;
}

extern "C" int nbm_batch_counts(nbm_ctx* ctx, void* stream, int32_t* counts, void* ws, size_t ws_bytes) {
  if (!ctx || !counts) return fail(NBM_EINVAL, "null argument");
  Layout pre = ctx->lo;
  pre.total = pre.prefix;   // only the bookkeeping is read
  int rc = check_ws(ctx, ws, ws_bytes, pre);
  if (rc) return rc;
  hipError_t e = launch_counts((hipStream_t)stream, at<Meta>(ws, ctx->lo.meta), counts);
  if (e != hipSuccess) return fail(NBM_EHIP, std::string("counts: ") + hipGetErrorString(e));
  return NBM_OK;
}
