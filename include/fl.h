/*
 * fl.h -- C-ABI of the MI355X (gfx950) finite-difference integral fractional
 * Laplacian library.
 *
 * Method: Duo & Zhang, "Accurate numerical methods for two and three
 * dimensional integral fractional Laplacian with applications"
 * (arXiv:1804.02718).  The operator (-Delta)^{alpha/2}, 0 < alpha < 2, on the
 * box (a, a + N h)^d, d = 1, 2 or 3, with u = 0 outside the box (the extended
 * homogeneous Dirichlet condition of Sec. 2), is discretised by the paper's
 * weighted-trapezoid scheme with splitting parameter gamma = 2 (the choice of
 * its Sec. 5): the 2D scheme of Sec. 2, the 3D scheme of Sec. 4, and the
 * one-dimensional case of the general-d scheme that Sec. 4 closes with (its
 * Theorems 3 and 4 hold for any d >= 1).  The stiffness matrix A is symmetric
 * positive definite multilevel Toeplitz (Toeplitz in 1D; Sec. 2 block form,
 * Sec. 4 three-level form) and is applied by circulant embedding and FFT.
 * The solves (Sec. 5.2 Poisson, Sec. 5.3 Allen-Cahn) run CG; by default
 * preconditioned by the sine-transform (tau) matrix of the same operator,
 * which is not part of the paper (fl_tau_apply, FL_SOLVE_TAU).
 *
 * Conventions shared by every call:
 *   - N >= 2 intervals per axis, n = N - 1 interior nodes per axis,
 *     M = n^d unknowns.  A grid vector holds the values at the interior nodes
 *     x_i = a + i h, i in [1, N-1]^d, flattened with the x index fastest (the
 *     ordering of the paper's matrix form).  Boundary and exterior values are
 *     0 and are not stored.  An operator built by fl_coeffs_box has its own
 *     node count per axis instead (fl_op_desc.nk) and M = their product.
 *   - Vector pointers are DEVICE pointers (hipMalloc'ed or torch CUDA
 *     tensors) owned by the caller; the library never frees them.  Host
 *     pointers are marked as such.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is ordered on that stream.  fl_apply returns without waiting for
 *     the GPU; the solvers return after convergence, with `info` filled.
 *   - An fl_op owns device workspaces: calls on one fl_op must not overlap
 *     (use one fl_op per concurrent stream).
 *   - Every call returns an fl_status; on error, fl_last_error() gives a
 *     message (per thread) and no output has been modified unless stated.
 */
#ifndef FL_H
#define FL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fl_op_s *fl_op;
typedef struct fl_unet_s *fl_unet;

typedef enum {
    FL_OK = 0,
    FL_E_INVAL = 1,       /* invalid argument (nothing changed)                  */
    FL_E_NOMEM = 2,       /* device allocation failed                            */
    FL_E_DEVICE = 3,      /* a HIP runtime error                                 */
    FL_E_NOCONV = 4,      /* iteration limit reached; output holds best iterate  */
    FL_E_BREAKDOWN = 5,   /* NaN/Inf or p^T A p <= 0 in CG                       */
    FL_E_UNSUPPORTED = 6  /* size outside the built kernel range                 */
} fl_status;

typedef enum { FL_FP64 = 0, FL_FP32 = 1 } fl_prec;

typedef enum {
    FL_SOLVE_AUTO = 0,    /* TAU, or TAU32 from 2^22 unknowns up, where it applies
                             (at most P/2 - 1 nodes per axis, i.e. every N but
                             2^k + 1, s0 + s1 lambda
                             > 0 on the sine modes; in the Allen-Cahn steps only
                             when 2 theta tau kappa A_ii > 0.5, else the system
                             is close to the identity); otherwise, Poisson:
                             REFINE for alpha <= 1.25, CG64 above (each
                             refinement step restarts CG, which costs the stiffer
                             operators more iterations than FP32 saves); the
                             Allen-Cahn steps: REFINE                            */
    FL_SOLVE_CG64 = 1,    /* plain conjugate gradients, FP64 matvec and vectors  */
    FL_SOLVE_REFINE = 2,  /* FP64 residual refinement around FP32-matvec CG      */
    FL_SOLVE_FPCG = 3,    /* flexible PCG with the learned preconditioner        */
    FL_SOLVE_TAU = 4,     /* flexible PCG, all FP64, with the sine-transform
                             (tau) preconditioner of the system matrix (see
                             fl_tau_apply); at most P/2 - 1 nodes per axis
                             (else FL_E_INVAL).  Falls back to CG64 like FPCG    */
    FL_SOLVE_TAU32 = 5    /* FP64 residual refinement around FP32 CG
                             preconditioned by the same sine transform in FP32
                             (inner tolerance 1e-4 unless inner_tol is set);
                             same operators as TAU.  AUTO takes it from 2^22
                             unknowns up, and falls back to TAU from the
                             current iterate if it fails                         */
} fl_solver;

typedef struct {
    int iters;            /* CG iterations (all inner iterations for REFINE)     */
    int outer_iters;      /* FP64 residual evaluations / refinement steps        */
    int fell_back;        /* 1 if the requested method gave up and a fallback
                             finished the solve from the current iterate: plain
                             FP64 CG after FPCG or TAU, TAU after TAU32         */
    int status;           /* fl_status of the solve                              */
    double relres;        /* final ||f - A u||_2 / ||f||_2, FP64 matvec          */
    double seconds;       /* host wall time of the call                          */
} fl_info;

typedef struct {
    int solver;           /* fl_solver                                           */
    int max_iter;         /* total CG iteration cap; <= 0 selects 50 M^{1/d}+1000 */
    int use_x0;           /* nonzero: u holds the initial guess on entry          */
    int check_every;      /* iterations between host convergence checks; <= 0 auto */
    double inner_tol;     /* REFINE: relative tolerance of each inner solve; <= 0 auto */
} fl_solve_opts;

typedef struct {
    int d, N, n, P, Q;    /* dimension, intervals, interior nodes, FFT length, P/2+1 */
    int64_t M;            /* unknowns nk[0] nk[1] nk[2] (n^d on the square)       */
    double alpha, h, c;   /* fractional order, mesh size, c_{d,alpha}            */
    double a0;            /* diagonal coefficient a_0 (A_ii = -c a_0)            */
    double gamma;         /* splitting parameter of the scheme                   */
    int nk[3];            /* interior nodes per axis, x first (1 past d)         */
} fl_op_desc;

/*
 * fl_coeffs -- build the operator for (d, alpha, h, N).
 * Computes on the GPU, in FP64: the element integrals of |xi|^{-(d+alpha-2)}
 * (Sec. 2 elements I_ij, Sec. 4 elements I_ijk), the coefficients a_v of the
 * scheme (Sec. 2 a_mn and a_00; Sec. 4 a_mns and a_000, the (1,1,1) origin
 * correction read as -1 times the origin element as the gamma = 2 limit rule
 * implies), the generator -c a_{|m|} of the Toeplitz matrix embedded in a
 * circulant of length P >= 2n - 1 per axis (a power of two, zeros in the gap),
 * and its FFT eigenvalues lambda (FP64 master, FP32 copy).
 *   d: 1, 2 or 3.  alpha: in (0, 2).  h > 0, finite.  N: 2 <= N <= 1025
 *   (d = 1), 2 <= N <= 8193 (d = 2), 2 <= N <= 513 (d = 3).  FFT lengths up
 *   to 2048 keep each line in LDS; 2D operators with N > 1025 (FFT length
 *   4096 to 16384, the paper's h = 2^-12 reference grid) run every radix pass
 *   over HBM: fl_apply and the single-operator solvers accept them;
 *   fl_apply_profiled, fl_autotune and fl_batch_create refuse them
 *   (FL_E_UNSUPPORTED) and they list no kernel variants.
 *   For d = 1 every element integral is one-dimensional, the correction of
 *   gamma = 2 moves the origin element's share to vertex 1, and a_0 =
 *   -sum_{m>=1} W_m / (m h)^2 - 2 L^{-alpha} / alpha.  *out receives a new handle (free with
 *   fl_op_destroy).  Uses the current HIP device; synchronises before
 *   returning.  Errors: FL_E_INVAL, FL_E_UNSUPPORTED, FL_E_NOMEM, FL_E_DEVICE.
 */
fl_status fl_coeffs(int d, double alpha, double h, int N, fl_op *out);

/*
 * fl_coeffs_gamma -- as fl_coeffs with the splitting parameter gamma of
 * Sec. 2 (the kernel |xi|^{-(d+alpha)} split into |xi|^{-gamma} on the
 * central difference quotient and the weight |xi|^{gamma-(d+alpha)}), gamma in
 * (alpha, 2].  gamma = 2 is fl_coeffs.  For gamma < 2 the origin limit of the
 * difference quotient is 0, so the origin-element corrections of a_mn
 * (weighted by floor(gamma/2)) vanish; the elements integrate
 * |xi|^{-(d+alpha-gamma)} and a_v = 2^sigma W_v / (2^d |xi_v|^gamma).  The
 * paper reports this choice as accurate to O(h^{2-alpha}) against O(h^2) for
 * gamma = 2 (Sec. 5.1, Example 5.1.2).  Errors as fl_coeffs; FL_E_INVAL when
 * gamma is outside (alpha, 2].
 */
fl_status fl_coeffs_gamma(int d, double alpha, double gamma, double h, int N, fl_op *out);

/*
 * fl_coeffs_box -- the operator on a box (a_x, b_x) x (a_y, b_y) [x (a_z, b_z)]
 * (Sec. 2 for d = 2, Sec. 4 for d = 3).  Nk[k] is the number of intervals of
 * width h along axis k (x first), the smallest with a_k + Nk[k] h >= b_k.  The
 * scheme takes L as the longest side and N = max Nk intervals along it, so
 * the coefficients a_v, v in [0, N]^d, and lambda are those of the square
 * (0, L)^d of fl_coeffs_gamma(d, alpha, gamma, h, N); the box keeps Nk[k] - 1
 * interior nodes per axis (the sums of the scheme stop at N_x - 1, N_y - 1,
 * N_z - 1), M = prod (Nk[k] - 1) unknowns, x index fastest.  Every call that
 * takes the handle works on the box's vectors of M entries, except the
 * learned-preconditioner solver (square grids only: FL_E_INVAL) and the
 * batched solver (which builds its own square operators).
 *   Nk: host array of d ints, each >= 2, max Nk within the range of
 *   fl_coeffs.  Errors as fl_coeffs_gamma; FL_E_INVAL when Nk is NULL or an
 *   entry is below 2.
 */
fl_status fl_coeffs_box(int d, double alpha, double gamma, double h, const int *Nk, fl_op *out);

/*
 * fl_apply -- y = A u, the discrete fractional Laplacian (Sec. 2 2D scheme /
 * Sec. 4 3D scheme), by zero-padded embedding, FFT, multiplication by lambda,
 * inverse FFT and crop.  prec = FL_FP64: u, y are double*; FL_FP32: float*.
 * u and y are device vectors of M entries and must not overlap.  Asynchronous
 * on `stream`.  Errors: FL_E_INVAL (null/overlap/prec), FL_E_DEVICE.
 */
fl_status fl_apply(fl_op op, const void *u, void *y, int prec, void *stream);

/*
 * fl_apply_noalloc -- fl_apply for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and kernel variant, with the spectra
 * workspaces taken from one static 64 MiB device array per GPU instead of the
 * operator's.  It calls no hipMalloc, hipFree or allocating routine; its
 * first call on a GPU looks up that GPU's copy of the array.  Every call on a
 * GPU shares the array, so calls that overlap in time on one GPU race; nothing
 * in it needs clearing between calls.  Arguments, layout and ownership as
 * fl_apply.  Errors: as fl_apply; FL_E_INVAL when the matvec's workspace
 * exceeds 64 MiB (it covers every 2D operator up to FFT length 2048, 3D up to
 * FFT length 256 in FP32 and 128 in FP64); FL_E_UNSUPPORTED for the large 2D
 * operators (FFT length above 2048).
 */
fl_status fl_apply_noalloc(fl_op op, const void *u, void *y, int prec, void *stream);

/*
 * fl_residual -- r = f - A u in FP64 (the residual of the Sec. 5.2 Poisson
 * problem), the FP64 matvec with f folded into its last pass.  f, u, r:
 * device double vectors of M entries; r may be f itself (each entry of f is
 * read before the same entry of r is written) but must not overlap u.
 * Asynchronous on `stream`.  Errors: FL_E_INVAL (null, u and r overlap),
 * FL_E_DEVICE.
 */
fl_status fl_residual(fl_op op, const double *f, const double *u, double *r, void *stream);

/*
 * fl_tau_apply -- z = M^{-1} r for the sine-transform (tau) preconditioner M of
 * K = s0 I + s1 A (s0, s1 >= 0, not both 0).  With P the embedding's FFT
 * length, the n' = P/2 - 1 nodes per axis make the sine vectors
 * sin(pi j k / (n' + 1)), k = 1..n', a basis; the tau matrix of K on them
 * (diagonal in that basis) has the circulant symbol of K at the frequencies
 * pi k / (n' + 1) as eigenvalues, i.e. K minus its two Hankel corrections
 * (for the Toeplitz levels of A: entries t_{i+j+2} and t_{2n'-i-j}).  On
 * power-of-two squares and cubes n' = n and M is that matrix; otherwise (other
 * N, boxes) M^{-1} is its inverse restricted to the operator's nodes, which
 * needs at most n' nodes per axis (every N but 2^k + 1).  Computed by the
 * matvec's passes on the odd extension of r with the symbol 1 / (s0 + s1
 * lambda), in FP64.  Not part of the paper's scheme: a preconditioner for its
 * CG solves (Sec. 5.2-5.3).
 * r, z: device double vectors of M entries, not overlapping.  The symbol is
 * rebuilt when (s0, s1) or the FP64 kernel variant change (a synchronising
 * step); then asynchronous on `stream`.  Errors: FL_E_INVAL (null, overlap,
 * s0/s1), FL_E_UNSUPPORTED (more than P/2 - 1 nodes on an axis),
 * FL_E_BREAKDOWN (s0 + s1 lambda not positive on a sine mode),
 * FL_E_NOMEM, FL_E_DEVICE.
 */
fl_status fl_tau_apply(fl_op op, const double *r, double *z, double s0, double s1,
                       void *stream);

/*
 * fl_poisson_solve -- solve A u = f (the fractional Poisson problem of
 * Sec. 5.2 with u = 0 outside the box) to ||f - A u||_2 <= tol ||f||_2,
 * checked with an FP64 residual.  f, u: device double vectors of M entries
 * (u is overwritten; the initial guess is 0).  Uses FL_SOLVE_AUTO.
 * tol > 0.  info (host, may be NULL) receives iteration counts and the
 * final FP64 relative residual.  Returns FL_E_NOCONV if the cap is reached
 * (u holds the last iterate), FL_E_BREAKDOWN on NaN/Inf.
 */
fl_status fl_poisson_solve(fl_op op, const double *f, double tol, double *u,
                           fl_info *info, void *stream);

/* As fl_poisson_solve, with explicit options (host pointer, may be NULL). */
fl_status fl_poisson_solve_ex(fl_op op, const double *f, double tol, double *u,
                              const fl_solve_opts *opts, fl_info *info, void *stream);

/*
 * fl_allen_cahn_step -- one semi-implicit step of
 *     u_t = -eps^2 (-Delta)^{alpha/2} u + u - u^3,  u = 0 outside the box,
 * Crank--Nicolson on the linear term (the time discretisation of Sec. 5.3),
 * the cubic term explicit:
 *     (I + tau eps^2 A / 2) u+ = u - tau eps^2 A u / 2 + tau (u - u^3),
 * solved with initial guess u by FL_SOLVE_AUTO (the sine-transform
 * preconditioned CG where it applies and pays, else FP32-matvec CG inside
 * FP64 residual refinement) to a relative FP64 residual of 1e-8.  u: device double vector
 * of M entries, updated in place.  tau > 0, eps > 0.
 */
fl_status fl_allen_cahn_step(fl_op op, double *u, double tau, double eps,
                             fl_info *info, void *stream);

/* As fl_allen_cahn_step with theta in (0, 1] weighting the implicit part
 * (theta = 1/2 Crank--Nicolson, theta = 1 backward Euler), solver tolerance
 * tol > 0 and solver choice (FL_SOLVE_AUTO, REFINE, CG64 or TAU). */
fl_status fl_allen_cahn_step_ex(fl_op op, double *u, double tau, double eps,
                                double theta, double tol, int solver,
                                fl_info *info, void *stream);

/*
 * fl_allen_cahn_step_gen -- one step of the general form
 *     u_t = -kappa (-Delta)^{alpha/2} u + gamma (w - w^3),  w = u - shift,
 * u = 0 outside the box, with the same theta-scheme on the linear term and
 * the explicit reaction term:
 *     (I + theta tau kappa A) u+ = u - (1-theta) tau kappa A u + tau gamma (w - w^3).
 * fl_allen_cahn_step_ex is kappa = eps^2, gamma = 1, shift = 0.  The
 * equation of Sec. 5.3 (u_t = -(-Delta)^{alpha/2} u - delta^{-alpha} u (u^2-1)
 * on (0,1)^d with u = -1 outside) is this form for ubar = u + 1, which is 0
 * outside: kappa = 1, gamma = delta^{-alpha}, shift = 1.  kappa >= 0 (0
 * leaves only the explicit reaction step), gamma and shift finite; other
 * arguments as in fl_allen_cahn_step_ex.
 */
fl_status fl_allen_cahn_step_gen(fl_op op, double *u, double tau, double kappa,
                                 double gamma, double shift, double theta,
                                 double tol, int solver, fl_info *info,
                                 void *stream);

/*
 * fl_apply_profiled -- fl_apply instrumented for measurement: runs `reps`
 * matvecs y = A u back to back on `stream`, each kernel launched with HIP
 * events recorded at its start and stop, synchronises, and writes the average
 * kernel time per pass in milliseconds to pass_ms (host, >= 5 floats) and the
 * number of passes (1 for d = 1: forward*lambda*inverse; 3 for d = 2:
 * X-forward, Y forward*lambda*inverse, X-inverse; 5 for d = 3: X-forward,
 * Y-forward, Z forward*lambda*inverse, Y-inverse, X-inverse) to *npass.  The result in y is that of fl_apply.
 */
fl_status fl_apply_profiled(fl_op op, const void *u, void *y, int prec, int reps, void *stream,
                            float *pass_ms, int *npass);

/*
 * Kernel variants.  Every (precision, FFT length, d) has one or more compiled
 * variants of the matvec kernels, differing in points per thread of the row
 * and strided passes (radix plan), spectrum tile width and rows per block;
 * variant 0 is the built-in default.  They all compute the same y = A u.
 *   fl_variant_count  -- number of variants for prec (host int).
 *   fl_variant_info   -- desc (host, 5 ints) = {row points per thread,
 *                        strided points per thread, tile width, row pairs per
 *                        block, kind}; kind 0: a workgroup per line block,
 *                        kind 1 (2D): one wavefront per FFT line, four rows per
 *                        row-pass workgroup.
 *   fl_select_variant -- use variant k for prec on this operator (synchronises).
 *   fl_autotune       -- time every variant (two rounds over the variants of
 *                        reps matvecs each, HIP events, on `stream`, scratch
 *                        vectors allocated and freed inside), select the
 *                        fastest, return its index in *best and, if
 *                        ms_per_variant (host, count floats) is non-null, each
 *                        variant's average milliseconds per matvec (the
 *                        smaller of its two rounds).
 */
fl_status fl_variant_count(fl_op op, int prec, int *count);
fl_status fl_variant_info(fl_op op, int prec, int k, int *desc);
fl_status fl_select_variant(fl_op op, int prec, int k);
fl_status fl_autotune(fl_op op, int prec, int reps, void *stream, int *best, float *ms_per_variant);

/*
 * fl_tune -- select the variant the on-disk tuning cache holds for this
 * operator's (d, FFT length, prec), timing every variant (fl_autotune, 10
 * matvecs each) and recording the fastest on a miss; its index in *variant
 * (host int).  The cache is the text file $FL_TUNE_CACHE, else
 * $HOME/.cache/fl_tune_gfx950.txt, one line per tuning; an empty
 * FL_TUNE_CACHE disables it (variant 0 is selected).  fl_batch_create takes
 * every class's variants from it.  Synchronises.  Errors: FL_E_INVAL,
 * FL_E_NOMEM, FL_E_DEVICE.
 */
fl_status fl_tune(fl_op op, int prec, int *variant);

/*
 * Batched fractional Poisson solves: `count` problems of the same dimension d
 * with their own N[i], alpha[i], h[i] (host arrays).
 *   fl_batch_create         -- builds every operator (as fl_coeffs; FFT length
 *                              <= 2048, i.e. 2D N <= 1025, else
 *                              FL_E_UNSUPPORTED) and groups
 *                              the problems into size classes of equal N; each
 *                              class runs all of its problems in every kernel
 *                              launch; one captured hipGraph holds a chunk
 *                              of inner CG iterations of every class (each on
 *                              its own branch) and is replayed in rounds of
 *                              1, 2, 4, ... with one host wait per round
 *                              (device done flags turn finished problems'
 *                              launches into no-ops).  Each class's kernel
 *                              variants come from the tuning cache (fl_tune).
 *                              A class whose N is
 *                              not 2^k + 1 and whose every problem has a
 *                              positive symbol on the sine modes preconditions
 *                              its inner CG by the sine transform (FP32, as
 *                              fl_tau_apply).
 *                              Synchronises.
 *   fl_batch_poisson_solve  -- solves A_i u_i = f_i to ||f_i - A_i u_i||_2 <=
 *                              tol ||f_i||_2 (FP64 residual refinement around
 *                              FP32 CG) for every i; f, u are host arrays of
 *                              `count` device pointers (double, M_i entries;
 *                              u overwritten, initial guess 0).  max_iter caps
 *                              each problem's inner iterations (<= 0: none).
 *                              infos (host, count entries, may be NULL) gets
 *                              each problem's result.  Work runs on internal
 *                              streams ordered after `stream`; `stream` waits
 *                              for the solutions.  Returns FL_E_NOCONV if any
 *                              problem missed the tolerance.
 *   fl_batch_info           -- number of size classes and the largest class.
 *   fl_batch_destroy        -- frees everything; NULL accepted.
 */
typedef struct fl_batch_s *fl_batch;
fl_status fl_batch_create(int d, int count, const int *N, const double *alpha, const double *h,
                          fl_batch *out);
fl_status fl_batch_poisson_solve(fl_batch b, const double *const *f, double *const *u, double tol,
                                 int max_iter, fl_info *infos, void *stream);
fl_status fl_batch_info(fl_batch b, int *nclasses, int *max_batch);
/* Of the last fl_batch_poisson_solve: the times the host waited for the GPU
 * and the replays of the all-class iteration graph; per class (host arrays of
 * nclasses ints, may be NULL) the FP32 and FP64 kernel variants in use. */
fl_status fl_batch_stats(fl_batch b, int *host_waits, int *graph_launches, int *var32, int *var64);
fl_status fl_batch_destroy(fl_batch b);

/*
 * Learned preconditioner: a convolutional U-Net (3 levels, 16/32/64 channels,
 * 3x3 bias-free convolutions with ReLU, 2x2 average pooling, nearest
 * upsampling with skip concatenation, 1x1 output) on an H x H grid, input
 * channels (r / rms(r), alpha), rms(r) = ||r|| / n over the n x n interior,
 * output an approximation of A^{-1} r / rms(r).
 * Convolutions run on bf16 MFMA with FP32 accumulation; weights are kept in
 * FP32 (Adam) with bf16 copies.  Not part of the paper's method: it feeds the
 * flexible PCG of FL_SOLVE_FPCG, which falls back to plain CG.
 *   fl_unet_create      -- H a multiple of 16 in [16, 2048], max_batch in
 *                          [1, 256] samples per step, seeded initialisation;
 *                          fp32_operands != 0 runs every GEMM on fp32
 *                          operands (v_mfma_f32_16x16x4_f32) instead of bf16,
 *                          a verification mode.
 *   fl_unet_step        -- nb samples: x (device, [nb][H][H][2] floats, NHWC),
 *                          y (device, [nb][H][H], may be NULL) receives the
 *                          output; with targets t (device, [nb][H][H]) also the
 *                          relative squared error per sample (loss_host) and
 *                          the weight gradients (grad_host, fl_unet_num_params
 *                          floats, may be NULL); lr > 0 takes one Adam step.
 *   fl_unet_pack        -- count training samples from device pairs
 *                          (r[z], sol[z]) of n x n doubles (host arrays of
 *                          device pointers; sol may be NULL): x[z] =
 *                          (r/rms(r), alpha[z]) and t[z] = sol/rms(r) on the
 *                          top-left n x n of the H x H grid, zero elsewhere.
 *   fl_unet_train       -- epochs over count device samples (x, t as in
 *                          fl_unet_step): seeded shuffle each epoch, batches
 *                          of `batch` (the ragged remainder is dropped), one
 *                          Adam step per batch with the learning rate
 *                          decaying from lr to lr_final on a cosine; mean
 *                          training loss per epoch to epoch_loss (host, may
 *                          be NULL).  ops NULL: relative L2 loss
 *                          ||y - t||^2 / ||t||^2 over the grid.  ops (host
 *                          array of count 2D operators, ops[i] the one whose
 *                          pair made sample i, n <= H): energy-norm loss
 *                          (y - t, A (y - t)) / (t, x0) on the interior, the
 *                          relative A-norm error of the preconditioned
 *                          residual (A t = x0 for an exact pair); one FP32
 *                          matvec per sample and step.  t NULL with ops:
 *                          the target-free residual loss
 *                          ||A y - x0||^2 / ||x0||^2 on the interior (A M
 *                          close to the identity on the inputs shown); two
 *                          FP32 matvecs per sample and step.
 *   fl_unet_get_weights / fl_unet_set_weights -- FP32 weights, layer by layer,
 *                          each [cout][(ky*ks + kx)*cin + ci] (host).
 *   fl_unet_apply       -- z = rms(r) Net(r/rms(r), alpha) for a residual r on
 *                          the n x n interior (device doubles, n <= H).
 *                          Asynchronous on `stream`: the norm of r and five
 *                          launches, each computing the two 3x3 convolutions
 *                          of one U-Net level (the last one also the 1x1 head
 *                          and the output scaling).  Calls on one network
 *                          share its workspaces: do not overlap them.
 *   fl_set_preconditioner -- attach (or detach with NULL) a network to a 2D
 *                          operator for FL_SOLVE_FPCG; not owned.
 *   fl_gemm_test        -- C = A B^T (host arrays [M][K], [N][K], [M][N];
 *                          M, N, K, kchunk multiples of 16) through the
 *                          network's GEMM kernel, operands rounded to bf16
 *                          (or fp32); kchunk < K takes the split-K path.
 */
fl_status fl_unet_create(int H, int max_batch, unsigned long long seed, int fp32_operands, fl_unet *out);
fl_status fl_unet_destroy(fl_unet u);
fl_status fl_unet_num_params(fl_unet u, long long *n);
fl_status fl_unet_step(fl_unet u, int nb, const float *x, const float *t, float *y, float lr,
                       float *loss_host, float *grad_host);
fl_status fl_unet_pack(fl_unet u, int count, const double *const *r, const double *const *sol, const double *alpha,
                       int n, float *x, float *t);
fl_status fl_unet_train(fl_unet u, long count, const float *x, const float *t, const fl_op *ops, int epochs,
                        int batch, float lr, float lr_final, unsigned long long seed, float *epoch_loss);
fl_status fl_unet_get_weights(fl_unet u, float *w_host);
fl_status fl_unet_set_weights(fl_unet u, const float *w_host);
fl_status fl_unet_apply(fl_unet u, const double *r, int n, double alpha, double *z, void *stream);
fl_status fl_set_preconditioner(fl_op op, fl_unet net);
fl_status fl_gemm_test(int M, int N, int K, int kchunk, int fp32_operands, const float *A_host, const float *B_host,
                       float *C_host);

/* Free the operator and its device workspaces.  NULL is accepted. */
fl_status fl_op_destroy(fl_op op);

/* Sizes and scalars of the operator (host struct). */
fl_status fl_op_describe(fl_op op, fl_op_desc *desc);

/* Copy a_v, v in [0,N]^d (x index fastest, a_host[0] = a_0) to the host
 * buffer a_host of (N+1)^d doubles. */
fl_status fl_get_coeffs(fl_op op, double *a_host);

/* Copy the FP64 eigenvalues lambda(k), k in [0,Q)^d (x index fastest; the
 * full spectrum is even in every axis), scaled by 1/P^d, to the host buffer
 * lam_host of Q^d doubles. */
fl_status fl_get_symbol(fl_op op, double *lam_host);

/* Human-readable name of a status code. */
const char *fl_status_string(fl_status s);

/* Message of the last error raised on the calling thread ("" if none). */
const char *fl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FL_H */
