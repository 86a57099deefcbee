/*
 * pbr.h -- C interface of libpbr, a GPU (MI355X, gfx950) implementation of the
 * parity-blocked rotated staggered discretisation of the Bloch elastic
 * eigenproblem
 *
 *     A_h(k) v = omega^2 M_h v,     A_h(k) = B_h(k) C_h B_h(k)^H
 *
 * (Sec. 3.3, Eq. 3.15).  B_h is assembled from four Bloch-periodic
 * body-diagonal differences (Eqs. 3.9-3.14), C_h is the nodewise 6x6 Voigt
 * stiffness (order [11,22,33,23,13,12], engineering shear; Sec. 2, Eq. 2.6) and
 * M_h = I_3 (x) diag(rho).  On even grids the problem splits into four parity
 * blocks (Theorem 4.1, Corollary 4.2); the library applies the operator, its
 * FFT-diagonal preconditioner, the shift-invert inner solve and the outer
 * Krylov eigensolver either in the full space or per block.
 *
 * CONVENTIONS (all calls)
 *   Grid        n1 x n2 x n3 nodes, node (i,j,k) has natural index
 *               i + n1*(j + n2*k) (i fastest; the Kronecker order of Eq. 3.5).
 *               Reduced spacings h_s = 1/n_s.
 *   Bloch k     kappa[3] in reduced reciprocal coordinates; boundary phases
 *               phi_l = 2*pi*kappa_l (Sec. 3.1, Eq. 3.3).
 *   Vectors     complex128, interleaved (re, im), component-major
 *               [v1 | v2 | v3]; each component has one entry per node.
 *   Blocks      block = -1 is the full space (3n unknowns); block = b in 0..3
 *               selects the parity block b = 2a + c, a = (i+j) mod 2,
 *               c = (j+k) mod 2, i.e. the paper's (sigma12, sigma13) =
 *               ((-1)^a, (-1)^(a+c)) (Sec. 4, Eqs. 4.2 and 4.11).  A block
 *               vector has 3n/4 entries; its node t = i + n1*(y2 + (n2/2)*y3)
 *               is the grid node (i, 2*y2 + o2, 2*y3 + o3) with
 *               o2 = (a+i) mod 2, o3 = (a+c+i) mod 2.  Blocks need even n1,n2,n3.
 *   Material    C21: n x 21 row-major doubles, per node the upper triangle of
 *               the symmetric Voigt matrix row by row (C11..C16, C22..C26, ...,
 *               C66), natural node order; rho: n doubles, all > 0.
 *   Lattice     A_lat: 3x3 column-major [a1|a2|a3] (NULL = identity); the
 *               Cartesian derivatives are D_m = sum_s (A_lat^-1)_{sm} Dhat_s
 *               (Sec. 3.3, Eq. 3.13).
 *   Eigenvalues lambda = omega^2, ascending.  f = sqrt(lambda)/(2 pi) is the
 *               caller's business.
 *
 * MEMORY AND STREAMS
 *   The caller owns every pointer it passes.  With on_device = 0 pointers are
 *   host memory, read or written before the call returns.  With on_device = 1
 *   they are device memory on the context's device, and the work is ordered on
 *   the context's stream (the caller synchronises before reading results; the
 *   library does not synchronise the stream except where a call must read a
 *   device scalar on the host, which the descriptions below say).  The context
 *   owns its device copies of the material and all work buffers; pbr_destroy
 *   frees them.
 *
 * ERRORS
 *   Every call returns a pbr_status and never throws.  A human-readable
 *   message for the last failing call on a context is returned by
 *   pbr_last_error(ctx) (pbr_last_error(NULL) for pbr_create failures).
 */
#ifndef PBR_H
#define PBR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbr_ctx pbr_ctx;

typedef enum pbr_status {
  PBR_OK = 0,
  PBR_EINVAL = -1,    /* bad argument: sizes, NaN/Inf or non-positive rho, nev, ... */
  PBR_EODDGRID = -2,  /* block >= 0 on a grid with an odd n_l (Theorem 4.1 needs even) */
  PBR_ENOMEM = -3,    /* device or host allocation failed */
  PBR_EDEVICE = -4,   /* a HIP runtime call failed */
  PBR_ENOCONV = -5,   /* iteration limit reached; partial results are written */
  PBR_ESTATE = -6     /* call made before pbr_set_material */
} pbr_status;

/* Solver settings (Sec. 7.1: tolerances 1e-12, 300 outer / 200 inner iterations). */
typedef struct pbr_opts {
  double tol;        /* outer: Ritz residual <= tol * |mu| of the shift-invert operator */
  double tol_inner;  /* inner PCG: ||r|| <= tol_inner * ||b|| (2-norm) */
  int maxit_outer;   /* maximum Krylov restarts */
  int maxit_inner;   /* maximum PCG iterations per solve */
  int ncv;           /* Krylov basis size; 0 = automatic (2*nev + 10, at most dim) */
  int precond;       /* 1 = FFT-diagonal preconditioner, 0 = none */
  int check_every;   /* PCG iterations between host convergence checks; 0 = automatic
                        (10).  The fused PCG (precond = 1) makes its first
                        check after about as many iterations as the context's previous
                        solve took; iterations past convergence change nothing. */
  int seed;          /* seed of the (deterministic) start vector */
  int concurrent;    /* pbr_eigs_merged / pbr_band_path: 1 = independent solves (the
                        four blocks, and up to 4 wave vectors of a path) advance in
                        lockstep, every kernel launch covering all of them; 0 = one
                        solve after another.  Results are identical. */
  int graphs;        /* 1 = each chunk of check_every PCG iterations is captured once
                        as a HIP graph (per k, shift and set of layouts) and replayed;
                        0 = kernels launched one by one.  Results are identical. */
  int warm_start;    /* pbr_eigs_merged / pbr_band_path: 1 = the Krylov start vector of a
                        solve is the sum of the Ritz vectors of the same layout at the
                        last wave vector of the previous group of 4 (or of its own
                        previous run when a block is re-solved with more eigenpairs),
                        plus a random part of half that norm; 0 = random start.  The
                        eigenvalues agree to the tolerance; fewer restarts along a path. */
} pbr_opts;

/* Statistics of one pbr_solve / pbr_eigs / pbr_eigs_merged / pbr_band_path call. */
typedef struct pbr_stats {
  int outer_iters;      /* Krylov restarts */
  int op_applies;       /* shift-invert applications (one PCG solve each) */
  int pcg_iters_total;  /* sum of PCG iterations */
  int pcg_iters_max;    /* largest PCG iteration count of one solve */
  int matvecs;          /* applications of A_h + s M_h (including final checks) */
  int n_zero;           /* Gamma null modes removed: 12 full space, 3 per block, else 0 */
  int converged;        /* eigenpairs (or 1 for a converged solve) delivered */
  int nev_block[4];     /* per-block nev used by pbr_eigs_merged (last k-point) */
  double pcg_avg;       /* pcg_iters_total / op_applies */
  double max_rel_resid; /* max ||A v - lambda M v|| / (||A v|| + |lambda| ||M v||) */
  double seconds;       /* host wall time of the call */
} pbr_stats;

/* Fill *o with the defaults: tol 1e-12, tol_inner 1e-12, maxit 300 / 200,
 * ncv automatic, precond 1, check_every automatic, seed 1, concurrent 1,
 * graphs 1, warm_start 1. */
void pbr_opts_default(pbr_opts *o);

/* Create a context for an n1 x n2 x n3 grid on HIP device `hip_device`.
 * hip_stream: a hipStream_t to order all work on, or NULL for a context-owned
 * stream.  A_lat: see CONVENTIONS.  Fails with PBR_EINVAL for n_l < 1 or a
 * singular A_lat, PBR_EDEVICE if the device cannot be used. */
pbr_status pbr_create(pbr_ctx **out, int n1, int n2, int n3, const double *A_lat,
                      int hip_device, void *hip_stream);

/* Upload the stiffness and density fields (layout in CONVENTIONS) and build the
 * per-block copies.  The preconditioner reference is reset to the volume means
 * of C and rho.  Fails with PBR_EINVAL on NaN/Inf entries or rho <= 0 (the check
 * reads the data on the host; device inputs are copied back for it). */
pbr_status pbr_set_material(pbr_ctx *c, const double *C21, const double *rho,
                            int on_device);

/* Storage form of the nodewise material C_h, rho (Eq. 3.15) that the operator
 * kernels read.  pbr_set_material always builds the dense form (21 stiffness
 * entries and rho per node).  When the material has at most 256 distinct
 * (C21, rho) rows, compared bit for bit, it also builds a palette form: the
 * distinct rows once, plus one byte per node naming its row.  Both forms hold
 * the same values: the operator's output (pbr_apply, pbr_apply_blocks) is
 * bit-identical either way, while solver results agree to rounding, since the
 * fused PCG sums its inner products per stencil tile and the two forms use
 * different tiles.  The palette form reads about a third of the bytes per
 * matvec.
 *
 * pbr_set_palette: enable = 1 (the default) lets the kernels read the palette
 * form whenever it exists; 0 makes them read the dense form.  Takes effect at
 * the next call, for the current and later materials.  PBR_EINVAL for a NULL
 * context or enable other than 0 or 1.
 *
 * pbr_material_palette: number of palette rows the kernels read (1..256), 0 when
 * they read the dense form (more than 256 distinct rows, or disabled), -1 for a
 * NULL context or before pbr_set_material. */
pbr_status pbr_set_palette(pbr_ctx *c, int enable);
int pbr_material_palette(const pbr_ctx *c);

/* Tile shape of the operator kernel (the fused matvec of Sec. 6.1 in pbr_apply,
 * pbr_apply_blocks and the solvers): ti x tj nodes of the (i, j) plane per
 * work-group.  ti = tj = 0 (the default) lets the autotuner choose per batch
 * size, box and material form, timing candidate shapes and chunk lengths on the
 * first launch; 16 x 13 (both forms) or 16 x 11 (palette form) pins that shape,
 * with only the chunk length tuned.  A pinned shape the current form does not
 * have is ignored for that form.  Operator outputs do not depend on the shape;
 * inner products of the fused PCG are summed per tile and may round
 * differently.  PBR_EINVAL for a NULL context or any other shape. */
pbr_status pbr_set_stencil_shape(pbr_ctx *c, int ti, int tj);

/* Pass structure of the FFT-diagonal preconditioner (pbr_precond and the fused
 * inner PCG) in a parity block: 0 (the default) or 3 = three passes over the
 * block vector where the block box has them (n1 = n2 with n1/2 one of 2, 3, 4,
 * 5, 6, 8, 10, 12, 15, 16, 20, 24, 30, 32, 40, 48, 64): both in-plane axes of a
 * plane at once, the third axis with the per-mode solves, the in-plane inverse;
 * 5 = five passes, one per axis and direction plus the solve (every other box,
 * and the full space, always uses five).  The two structures compute the same
 * operator (Sec. 5.1-5.4) and agree to rounding.  Takes effect at the next
 * call.  PBR_EINVAL for a NULL context or another value. */
pbr_status pbr_set_precond_passes(pbr_ctx *c, int passes);

/* i-width of the mode-solve pass of the three-pass block preconditioner (the
 * third-axis transforms and per-mode 3 x 3 solves of Sec. 5.3-5.4): bi
 * consecutive i-values of both sub-lattices per work-group.  0 (the default)
 * lets the autotuner choose per box and batch size (timed on a copy of the
 * data at the first call); 8, 16 or 32 pins that width where it divides n1 (a
 * width that does not is ignored).  The operator does not depend on the width;
 * the (r, z) partials of the fused PCG are summed per work-group and may round
 * differently.  PBR_EINVAL for a NULL context or any other value. */
pbr_status pbr_set_solve_width(pbr_ctx *c, int bi);

/* Override the constant reference material of the preconditioner
 * (K(m) = Bhat(m) C_ref Bhat(m)^H + shift * rho_ref * I_3, Sec. 5.3-5.4): C21_ref
 * is 21 host doubles in the C21 order, rho_ref > 0. */
pbr_status pbr_set_reference(pbr_ctx *c, const double *C21_ref, double rho_ref);

/* delta = 0.30 * C_max, C_max the largest |C_pq| of the material (Eq. 7.7).
 * Returns a negative value before pbr_set_material. */
double pbr_default_shift(const pbr_ctx *c);

/* Number of complex unknowns: 3n for block = -1, 3n/4 for a block; -1 on
 * error (bad block or odd grid). */
long pbr_block_dim(const pbr_ctx *c, int block);

/* y = Q_b^* full (gather) and full = Q_b y on block b's entries (scatter; the
 * other entries of full are left untouched) -- Corollary 4.2, Eq. 4.14. */
pbr_status pbr_block_gather(pbr_ctx *c, int block, const void *full, void *blk,
                            int on_device);
pbr_status pbr_block_scatter(pbr_ctx *c, int block, const void *blk, void *full,
                             int on_device);

/* y = (A_h(k) + s M_h) x in the full space (block = -1) or restricted to a
 * parity block (A_sigma + s M_sigma, Eq. 4.14), matrix-free as
 * x -> B^H x -> C B^H x -> B C B^H x (Sec. 6.1).  x and y must not overlap.
 * Size limit (32-bit buffer offsets in the kernel): one layout's vector (48 B
 * per node) and its stiffness tiles (176 B per node, runs of 16 nodes along n1)
 * must each stay below 2 GiB: a cube up to n = 225 in the full space and up to
 * n = 364 in the parity blocks (a block holds a quarter of the nodes); larger
 * grids get PBR_EINVAL from this call and from every call that applies the
 * operator (pbr_apply_blocks, pbr_solve, the eigensolvers, pbr_eig_grad). */
pbr_status pbr_apply(pbr_ctx *c, const double kappa[3], int block, double s,
                     const void *x, void *y, int on_device);

/* y_b = (A_sigma(b) + s M_sigma(b)) x_b for all four parity blocks in one
 * launch: the block-diagonal form of A_h(k) + s M_h in the parity-block basis
 * (Theorem 4.1, Corollary 4.2).  x and y hold the four block vectors back to
 * back, block 0 first, each 3n/4 complex in the block layout of CONVENTIONS
 * (3n complex in all).  Even grids only (PBR_EODDGRID otherwise); x and y must
 * not overlap. */
pbr_status pbr_apply_blocks(pbr_ctx *c, const double kappa[3], double s, const void *x,
                            void *y, int on_device);

/* z = T_xi diag_m(K(m)^-1) T_xi^H r with K(m) = Bhat(m) C_ref Bhat(m)^H +
 * shift * rho_ref * I_3: the FFT-diagonal preconditioner of the shifted system
 * (Fourier bases of Sec. 5.1-5.2, symbols Eqs. 5.8-5.11; T_xi = T full,
 * T_sigma = T F_sigma for a block).  shift > 0.  Every transform length (n_l
 * in the full space, n_l / 2 in a block) must be one of 1, 2, 3, 4, 5, 6, 8, 10,
 * 12, 15, 16, 20, 24, 30, 32, 40, 48, 60, 64, 80, 96, 120, 128, 160, 192, 240,
 * 256 (PBR_EINVAL otherwise); the same holds for pbr_solve, pbr_eigs and the
 * calls built on them with the preconditioner on. */
pbr_status pbr_precond(pbr_ctx *c, const double kappa[3], int block, double shift,
                       const void *r, void *z, int on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pbr_precond
 * on device pointers with no allocation of any kind.  Same arguments, kernels
 * and result as pbr_precond with on_device = 1 (bit for bit); r and z are device
 * memory on the context's device, work is ordered on the context's stream.
 * The per-wave-vector tables the kernels read (roots, twists, mode phases of the
 * three axes, and for a block the mode phases in the order of its three-pass
 * transforms) are written by each call into a fixed array of 12 x 256 complex128
 * (49,152 bytes) that every device the library runs on holds until the process
 * ends, set up by pbr_create; hence every n_l must be at most 256 (PBR_EINVAL
 * otherwise, before any work).  The array is shared by all contexts on a device
 * and keeps the last call's contents: calls that overlap in time on one device
 * (other streams, other host threads) race on it and must be serialised by the
 * caller.  Where pbr_precond tunes a kernel's work split at its first call on a
 * box, this call uses the split the context has tuned, or the default one, and
 * matches pbr_precond bit for bit once pbr_precond has run on that box.
 * PBR_ESTATE before pbr_set_material. */
pbr_status pbr_precond_noalloc(pbr_ctx *c, const double kappa[3], int block, double shift,
                               const void *r, void *z);

/* Solve (A_h(k) + shift M_h) x = b (block: A_sigma, M_sigma) by preconditioned
 * conjugate gradients from x = 0 (the inner solve of Sec. 6.1, Eq. 6.2).  Reads
 * the residual norm on the host every opts->check_every iterations.  Returns
 * PBR_ENOCONV (x holds the last iterate) if opts->maxit_inner is reached. */
pbr_status pbr_solve(pbr_ctx *c, const double kappa[3], int block, double shift,
                     const void *b, void *x, const pbr_opts *opts, pbr_stats *st,
                     int on_device);

/* nev lowest eigenvalues of (A_h(k), M_h) (block = -1) or of block b
 * (Corollary 4.2), by a thick-restart Lanczos (Krylov-Schur) iteration on the
 * shift-invert operator (A + shift M)^-1 M (Sec. 6.1), each application being a
 * pbr_solve.  shift <= 0 selects pbr_default_shift.  At the Gamma point (every
 * kappa_l an integer) the zero-derivative modes chi_mu e_alpha (Sec. 6.2,
 * Appendix C) are projected out and the nev lowest non-zero eigenvalues are
 * returned; st->n_zero reports how many null modes were removed.
 * evals: nev host doubles.  evecs: NULL, or dim x nev complex128 column-major
 * (on the host if evecs_on_device = 0), M-normalised (v^H M v = 1).
 * Fails with PBR_EINVAL if nev < 1 or nev + n_zero >= dim. */
pbr_status pbr_eigs(pbr_ctx *c, const double kappa[3], int block, int nev,
                    double shift, const pbr_opts *opts, double *evals, void *evecs,
                    int evecs_on_device, pbr_stats *st);

/* nev lowest eigenvalues of the full pencil obtained by solving the four parity
 * blocks and merging their spectra (Sec. 6.1).  Each block starts with
 * nev_b = ceil(nev/4) + 1 eigenpairs; a block whose largest computed eigenvalue
 * lies below the merged nev-th value is recomputed with more eigenpairs until
 * every block certifies the cut (at most 8 rounds); PBR_ENOCONV, with the
 * merged values written, when a block stays uncertified.  Needs an even grid. */
pbr_status pbr_eigs_merged(pbr_ctx *c, const double kappa[3], int nev, double shift,
                           const pbr_opts *opts, double *evals, pbr_stats *st);

/* pbr_eigs_merged with the eigenvectors: the nev lowest eigenpairs of the full
 * pencil from the four parity blocks (Corollary 4.2, same certification rule).
 * evals: nev host doubles, ascending.  blocks: nev host ints, the parity block
 * each eigenpair comes from (values equal across blocks are ordered by block).
 * evecs: nev vectors of pbr_block_dim(c, 0) complex128 one after another
 * (device memory if evecs_on_device, else host), vector t in block blocks[t]'s
 * layout, M-normalised (v^H M_sigma v = 1); pbr_block_scatter places one in the
 * full space.  These are the per-block pairs pbr_eig_grad takes. */
pbr_status pbr_eigs_merged_vecs(pbr_ctx *c, const double kappa[3], int nev, double shift,
                                const pbr_opts *opts, double *evals, int *blocks, void *evecs,
                                int evecs_on_device, pbr_stats *st);

/* Band structure along nk reduced wave vectors kappas (nk x 3 row-major host
 * doubles): evals[q*nev + t] is the t-th eigenvalue at kappa q.  blocked = 1
 * gives pbr_eigs_merged's result at every point, blocked = 0 the full-space
 * pbr_eigs'.  With opts->concurrent the path is processed 4 wave vectors at a
 * time, all their solves in lockstep (16 block solves, or 4 full-space ones,
 * per kernel launch).  st (optional) accumulates over the path. */
pbr_status pbr_band_path(pbr_ctx *c, int nk, const double *kappas, int nev,
                         int blocked, double shift, const pbr_opts *opts,
                         double *evals, pbr_stats *st);

/* Band structures of several unit cells at once, each with its own grid,
 * lattice and material (one context per cell; the method is the per-cell one of
 * pbr_band_path, Sec. 6.1).  Cell q is ctxs[q] with nk[q] reduced wave vectors
 * kappas[q] (nk[q] x 3, host, row-major) and results evals[q] (nk[q] x nev,
 * host); shift <= 0 takes each cell's default.  The cells' paths run
 * concurrently, one native host thread per cell driving its context's own
 * stream, so that small cells fill the GPU together; every cell's eigenvalues
 * are bit for bit those of pbr_band_path on it in the same state.  (A context's
 * autotuners pick the operator's tile shape and the mode-solve width by timing
 * at its first launch of each shape of batch, and those choices group the PCG
 * inner products; first calls timed under different load can choose
 * differently.  pbr_set_stencil_shape and pbr_set_solve_width pin them.)  The
 * contexts must be distinct,
 * on one device, and must not share a stream; 1 <= ncells <= 64.  st (optional)
 * receives ncells statistics.  Returns PBR_OK, or the first failing cell's
 * status (its message via pbr_last_error on that context; every cell is run);
 * PBR_EINVAL for bad arguments before any cell starts. */
pbr_status pbr_band_paths(int ncells, pbr_ctx *const *ctxs, const int *nk,
                          const double *const *kappas, int nev, int blocked,
                          double shift, const pbr_opts *opts, double *const *evals,
                          pbr_stats *st);

/* Derivatives of eigenvalues with respect to the material (first-order
 * perturbation of the pencil of Eq. 3.15): for nvec eigenpairs (lambda[s], v_s)
 * of layout `block` at kappa, with v_s^H M v_s = 1 as pbr_eigs returns them,
 * ADDS sum_s weight[s] * d lambda_s / d C21 to gC21 (n x 21, natural order and
 * the C21 entry order of CONVENTIONS) and sum_s weight[s] * d lambda_s / d rho
 * to grho (n):
 *   d lambda / d C21_(a,b)(x) = |e_a(x)|^2 (a = b), 2 Re(conj(e_a) e_b) (a < b),
 *   d lambda / d rho(x) = -lambda |v(x)|^2,
 * with the strains e = B_h^H v recomputed from v.  A single derivative is
 * defined for a simple eigenvalue; for a cluster of equal eigenvalues pass an
 * orthonormal basis of the cluster with equal weights (the sum is defined).
 * evecs: nvec vectors of pbr_block_dim(c, block) complex, one after another;
 * lambda, weight: host arrays.  Block derivatives vanish off the block's nodes. */
pbr_status pbr_eig_grad(pbr_ctx *c, const double kappa[3], int block, int nvec,
                        const double *lambda, const double *weight, const void *evecs,
                        int evecs_on_device, double *gC21, double *grho, int grad_on_device);

/* The HIP stream (hipStream_t) the context orders its work on: the one given
 * to pbr_create, or the context's own stream (created with default flags, so
 * HIP orders it against the legacy null stream: work a caller issues on the
 * null stream before a call runs before the call's kernels, and work issued
 * after it runs after them).  NULL for a NULL context.  Callers time the
 * library's kernels with events recorded on this stream. */
void *pbr_stream(const pbr_ctx *c);

/* Measurement support, not an operation of the method: copy `bytes` (a
 * multiple of 16) from src to dst, both device memory on the context's device,
 * with a plain streaming kernel on the context's stream (16-byte non-temporal
 * loads and stores, no reuse).  Its rate is the copy reference the operator
 * kernels' HBM rates are compared with.  PBR_EINVAL for NULL pointers or a bad
 * byte count; src and dst must not overlap. */
pbr_status pbr_copy_probe(pbr_ctx *c, const void *src, void *dst, long bytes);

/* Message of the last failing call on c (or of the last failing pbr_create when
 * c is NULL).  The string lives until the next call on c. */
const char *pbr_last_error(const pbr_ctx *c);

/* Free the context and all its device memory.  NULL is ignored. */
void pbr_destroy(pbr_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* PBR_H */
