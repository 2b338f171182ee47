/*
 * nbm.h — C ABI of the MI355X (gfx950) Neural Bootstrapping Method library.
 *
 * The Neural Bootstrapping Method (paper: "Neuro-Symbolic Partial Differential
 * Equation Solver", Sec. 3) trains two networks u^- and u^+, one per side of a
 * level-set interface, by minimising the locally preconditioned residual of a
 * finite-volume discretisation of the interface problem of Sec. 2,
 *     k u - div(mu grad u) = f in Omega^+-,  [u] = alpha, [mu d_n u] = beta on Gamma,
 * evaluated on implicit cells centred at random collocation points, with
 * automatic differentiation through the residual kernels and Adam.
 * The paper's loss equation is missing from its text; the residual computed
 * here is this library's cut-cell reading of it (vertex-centred cell of
 * side h at each point, face/volume fractions of the piecewise-linear level
 * set, jump extension J = alpha + dist * [d_n u], Jacobi preconditioning,
 * loss = mean of squared point residuals, interior and boundary points).
 *
 * Conventions shared by every entry point
 *   - Device memory is owned by the caller (e.g. torch tensors passed as raw
 *     pointers).  The library owns only the host-side context; it never
 *     allocates device memory.  Every pointer marked "device" must point to
 *     memory on the current HIP device.
 *   - Every call is asynchronous on the given stream and never synchronises
 *     the device.  A NULL stream means the default stream.
 *   - Return 0 on success or a negative NBM_E* code.  Arguments are validated
 *     before any launch; on error nothing is enqueued and nbm_last_error()
 *     describes the problem.  No C++ exception crosses the ABI.
 *   - NaN/Inf propagate.  If a batch holds more cut cells than the context's
 *     cut capacity, the loss is written as NaN.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Parameters are FP32, packed net^- then net^+; per net: W1[W][d], b1[W],
 *     then for l = 2..L: W_l[W][W], b_l[W], then w_out[W], b_out (matrices
 *     row-major, row = output neuron).
 *   - Points are FP32 [n][d] row-major.  Interior points must lie in
 *     [-1+h, 1-h]^d, boundary points on the faces of [-1,1]^d.
 */
#ifndef NBM_H
#define NBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBM_OK 0
#define NBM_EINVAL -1       /* invalid argument or configuration */
#define NBM_EWORKSPACE -2   /* workspace missing, too small, or not prepared */
#define NBM_EUNSUPPORTED -3 /* configuration not compiled into this library */
#define NBM_EHIP -4         /* a HIP runtime call failed */

#define NBM_ACT_TANH 0
#define NBM_ACT_SIN 1
#define NBM_PREC_FP32 0     /* FP32 MFMA operands, FP32 accumulation */
#define NBM_PREC_BF16 1     /* BF16 MFMA operands, FP32 accumulation */
#define NBM_IFACE_SPHERE 0  /* |x| - radius (circle in 2-D) */
#define NBM_IFACE_STAR 1    /* |x| - radius - amp sin(5 theta) sin(4 psi) */
#define NBM_IFACE_PLANE 2   /* plane_n . x - plane_c */
#define NBM_IFACE_MESH 3    /* level set stored on a coarse mesh (paper Sec. 3), multilinear */
#define NBM_PROB_MMS_2D 0   /* u^- = exp(x+y), u^+ = sin(pi x) cos(pi y) */
#define NBM_PROB_MMS_SPHERE 1 /* u^- = exp(z), u^+ = cos x sin y (paper Sec. 4.1) */
#define NBM_PROB_FOURIER 2  /* f^- = f^+ = sum_k a_k cos(pi k.x) + b_k sin(pi k.x) */
#define NBM_PROB_LINEAR 3   /* u^- = a.x + a0, u^+ = b.x + b0 */
#define NBM_MU_CONST 0      /* mu^-+ = mu_minus, mu_plus */
#define NBM_MU_PAPER 1      /* mu^- = y^2 ln(x+2) + 4, mu^+ = exp(-z) (paper Sec. 4.1) */

/* Problem and network description (paper Sec. 2 problem statement; Sec. 3
 * two networks; Sec. 4.1 workload).  Host memory, copied by nbm_create. */
typedef struct nbm_config {
  int32_t dim;        /* 2 or 3 */
  int32_t width;      /* W, hidden width */
  int32_t depth;      /* L >= 2 hidden layers (L-1 hidden->hidden matrices) */
  int32_t act;        /* NBM_ACT_* */
  int32_t prec;       /* NBM_PREC_* */
  double h;           /* implicit cell spacing, a power of two in [2^-20, 2^-2] */
  int32_t interface_kind; /* NBM_IFACE_* */
  double radius;      /* sphere / star radius */
  double star_amp;    /* star amplitude */
  double plane_n[3];  /* plane normal (unit) */
  double plane_c;     /* plane offset */
  double mu_minus, mu_plus; /* piecewise-constant diffusion coefficients > 0; with
                               NBM_MU_PAPER they only tell which side is smaller */
  int32_t mu_kind;    /* NBM_MU_*: with NBM_MU_PAPER every face takes mu at its centre
                         (the step then runs the layered kernels) */
  double k_minus, k_plus;   /* Helmholtz coefficients k^-+ >= 0 of the term k u */
  int32_t problem;    /* NBM_PROB_* */
  double alpha_const, beta_const; /* jump data of NBM_PROB_FOURIER */
  double lin_a[4], lin_b[4];      /* NBM_PROB_LINEAR coefficients */
  int32_t n_modes;    /* NBM_PROB_FOURIER: number of modes */
  const int32_t* mode_k; /* host [n_modes][3] integer wave vectors */
  const double* mode_a;  /* host [n_modes] cosine amplitudes */
  const double* mode_b;  /* host [n_modes] sine amplitudes */
  int64_t max_points;    /* largest interior batch n the workspace must hold */
  int64_t max_boundary;  /* largest boundary batch nb */
  int64_t cut_capacity;  /* max cut cells per batch; 0 -> max_points/8 + 64 */
  int32_t eval_only;     /* 1: workspace for nbm_eval only (max_points = largest
                            query tile); training calls return NBM_EWORKSPACE */
  int32_t phi_n;         /* NBM_IFACE_MESH: intervals per axis of the level-set mesh
                            over [-1,1]^dim, 2..1024 */
  const double* phi_table; /* NBM_IFACE_MESH: host [(phi_n+1)^dim] nodal values at
                            -1 + 2 j / phi_n, axis 0 fastest; copied by nbm_create,
                            placed in the workspace by nbm_prepare */
  int32_t levels;        /* implicit refinement levels beyond the base (paper
                            Sec. 3 implicit cells at several resolutions, Sec. 4.2
                            base resolution refined implicitly): every point
                            carries cells of side h, h/2, ..., h/2^levels and the
                            loss is the sum of the levels' losses.  0..6,
                            h/2^levels >= 2^-20 */
} nbm_config;

typedef struct nbm_ctx nbm_ctx;

/* Validate cfg and create a host-side context.  No device work. */
int nbm_create(const nbm_config* cfg, nbm_ctx** out);
void nbm_destroy(nbm_ctx* ctx);

/* Number of FP32 parameters (both networks). */
int64_t nbm_param_count(const nbm_ctx* ctx);

/* Device workspace bytes a call needs for a batch of n interior and nb
 * boundary points (nbm_forward_residual, nbm_backward), or for n queries
 * (nbm_eval, nb = 0).  A workspace sized for (n, nb) serves every smaller
 * batch.  Returns 0 if n > max_points, nb > max_boundary or either is
 * negative.  The caller allocates it (256-byte aligned) and owns it. */
size_t nbm_workspace_bytes(const nbm_ctx* ctx, int64_t n, int64_t nb);

/* Copy the problem tables (Fourier modes, level-set mesh) into the front of the workspace
 * (the part whose offsets do not depend on the batch size).  Must be called
 * once for each workspace before the other workspace-using calls; blocks the
 * host until the copy is done. */
int nbm_prepare(nbm_ctx* ctx, void* stream, void* ws, size_t ws_bytes);

/* Random collocation points (paper Sec. 3: residuals minimised on randomly
 * sampled points).  Philox4x32-10, interior point i of step s uses counter
 * (i, s_lo, s_hi, 0), boundary point b (b, s_lo, s_hi, 1), key = seed.
 * Interior points on the 2^-22 lattice in [-1+h, 1-h]^d, boundary points on
 * the lattice of the faces of [-1,1]^d.  pts [n][d], bpts [nb][d] device. */
int nbm_sample_points(nbm_ctx* ctx, void* stream, uint64_t seed, int64_t step, float* pts,
                      int64_t n, float* bpts, int64_t nb);

/* Forward pass: residual of every interior and boundary point and the loss
 * L = (sum_p r_p^2 + sum_b r_b^2) / (n + nb), accumulated in FP64
 * (paper Sec. 3: point residuals r_p = |M^-1 A u - M^-1 b| aggregated into a
 * global loss); with levels > 0, L = sum over levels l of the loss of cells
 * of side h / 2^l.  params [P] device; pts [n][d], bpts [nb][d] device;
 * residual [(levels + 1) (n + nb)] device (level-major) or NULL; loss: one
 * device double.
 * If grad is not NULL the same pass also writes dL/dtheta [P] (FP32, reduced
 * in FP64 in a fixed order): the fused forward + residual + backward step. */
int nbm_forward_residual(nbm_ctx* ctx, void* stream, const float* params, const float* pts,
                         int64_t n, const float* bpts, int64_t nb, float* residual,
                         double* loss, float* grad, void* ws, size_t ws_bytes);

/* Allocation-free form of nbm_forward_residual, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  Same arguments and
 * results as nbm_forward_residual without the workspace: the step runs in a
 * static device array of NBM_SCRATCH_BYTES (64 MiB) that the library holds on
 * each GPU it runs on until the process ends; no call allocates or frees.
 * Returns NBM_EWORKSPACE if the batch's workspace (nbm_workspace_bytes(ctx,
 * n, nb)) exceeds NBM_SCRATCH_BYTES -- the 64-wide and 16-wide networks fit
 * up to their full training batches, the 128-wide ones do not -- and
 * NBM_EUNSUPPORTED for the Fourier problem (its tables live in a prepared
 * workspace).  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (two streams, two
 * threads, two contexts) race and must be serialised by the caller.
 * nbm_batch_counts does not see this entry point's batches. */
#define NBM_SCRATCH_BYTES (64ull << 20)
int nbm_forward_residual_noalloc(nbm_ctx* ctx, void* stream, const float* params, const float* pts,
                                 int64_t n, const float* bpts, int64_t nb, float* residual,
                                 double* loss, float* grad);

/* Backward pass (paper Sec. 3: automatic differentiation across the NBM
 * kernels): recomputes the forward pass and writes dL * dL/dtheta into
 * grad [P] (device FP32).  Holds no state between calls. */
int nbm_backward(nbm_ctx* ctx, void* stream, const float* params, const float* pts, int64_t n,
                 const float* bpts, int64_t nb, double dL, float* grad, void* ws,
                 size_t ws_bytes);

/* Adam (paper Sec. 3), bias-corrected, FP32, in place on params, m, v [P]
 * (device); grad [P] device; step is 1-based. */
int nbm_adam_step(nbm_ctx* ctx, void* stream, float* params, float* m, float* v,
                  const float* grad, int64_t step, float lr, float beta1, float beta2,
                  float eps);

/* Evaluate the surrogate u(x) = u^{sigma(x)}(x) (network of the side of x).
 * With query != NULL: query [m][d] device points.  With query == NULL: the
 * points of tile `tile_index` of the grid_n^d lattice x = -1 + 2 i / grid_n
 * (i = 0..grid_n-1 per axis, axis 0 fastest, tiles of m consecutive points)
 * are generated in the kernel.  u_out [m] device FP32.  m <= max_points. */
int nbm_eval(nbm_ctx* ctx, void* stream, const float* params, const float* query, int64_t m,
             int64_t tile_index, int32_t grid_n, float* u_out, void* ws, size_t ws_bytes);

/* Grid fallback of the evaluation: where the surrogate's error against the
 * grid solution (the method without the learned part) exceeds a stated
 * tolerance, a tile takes the grid solution instead.  Writes, at the m points
 * of tile `tile_index` of the grid_n^d lattice (as nbm_eval with query ==
 * NULL), the multilinear interpolation of U, the solution on the
 * (judge_n + 1)^d nodes -1 + 2 j / judge_n (device FP64, axis 0 fastest).
 * u_out [m] device FP32.  No workspace; U is only read. */
int nbm_grid_interp(nbm_ctx* ctx, void* stream, const double* U, int32_t judge_n, int64_t tile_index,
                    int32_t grid_n, int64_t m, float* u_out);

/* Classes of the last batch seen by nbm_forward_residual / nbm_backward on
 * this workspace, written to counts[8] (device int32): interior A^-, A^+,
 * cut, boundary^-, boundary^+, overflow flag, fallback flag, 0.  The
 * fallback flag is 1 when the 128-wide forward/backward with BF16 operands
 * met an activation argument beyond its fast (micro-series) form and
 * recomputed the batch with per-element series tiers (same results; the
 * second pass costs time).  FP32 operands always take the per-element form. */
int nbm_batch_counts(nbm_ctx* ctx, void* stream, int32_t* counts, void* ws, size_t ws_bytes);

/* Measurement support.  With timing enabled, every later call records a
 * pair of HIP events on its stream around each kernel group:
 * 0 shadow+classify+compact, 1 forward streams, 2 residual+loss,
 * 3 backward (the fused forward/residual/backward launch, or one pair per
 * hidden-layer launch of the layered path), 4 gradient reduction, 5 Adam,
 * 6 sampling, 7 evaluation, 8 weight-gradient launches of the 128-wide
 * two-pass backward (one pair per hidden layer), 9 Fourier forcing.
 * Costs a little host time per call. */
#define NBM_TIMING_GROUPS 10
int nbm_set_timing(nbm_ctx* ctx, int enable);

/* Wait for the recorded events, write per group the summed milliseconds
 * ms[NBM_TIMING_GROUPS] and the number of timed launches
 * launches[NBM_TIMING_GROUPS] (host arrays), then forget the records.
 * Blocks the host. */
int nbm_read_timing(nbm_ctx* ctx, double* ms, int64_t* launches);

/* Thread-local description of the last error. */
const char* nbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NBM_H */
