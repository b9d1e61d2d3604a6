/*
 * sgm.h -- C ABI of libsgm, a gfx950 (MI355X) implementation of the
 * data-parallel hot path of the spectral Galerkin method in tensor-product
 * domains with one non-periodic (Chebyshev/Shen) direction and one or two
 * periodic (Fourier) directions (Mortensen, "Shenfun - automating the
 * spectral Galerkin method").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are DEVICE pointers owned by the caller.  Real data
 *   are IEEE binary64; complex data are interleaved (re, im) binary64 pairs.
 * - Every call is asynchronous on the given stream (a hipStream_t passed as
 *   void*, NULL = the null stream).  Plans, GL batches and networks own their
 *   workspace and tables, allocated at creation; the transform, solve and
 *   time-step calls allocate nothing (sgm_fno_advance_checked sizes its
 *   workspace on its first call, as documented there).
 * - Return value: SGM_OK (0) or a negative SGM_ERR_* code; a human-readable
 *   detail for the last failing call of the calling thread is available from
 *   sgm_last_error().  No C++ exception crosses this boundary.
 * - Physical arrays are C-ordered [x][y] or [x][y][z] with z contiguous; x
 *   holds the N Gauss-Chebyshev points x_j = cos((2j+1) pi / (2N)) (Sec. 3.4.2),
 *   y and z the uniform periodic grids 2 pi k / M (Sec. 3.4.1).
 * - Spectral arrays are C-ordered [l][m] or [l][m][n]: N rows along x (rows
 *   l >= the number of basis functions are written as zero), the Fourier
 *   axes in FFT order (0..ceil(M/2)-1, then -floor(M/2)..-1; eq. wavenumber_even);
 *   an R2C last axis keeps n = 0..M/2 (Sec. 3.4.1, Hermitian symmetry).
 */
#ifndef SGM_H
#define SGM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int sgm_status;
#define SGM_OK 0
#define SGM_ERR_INVALID_ARG (-1)
#define SGM_ERR_UNSUPPORTED_SIZE (-2)
#define SGM_ERR_HIP (-3)
#define SGM_ERR_OOM (-4)
#define SGM_ERR_UNIMPLEMENTED (-5)
#define SGM_ERR_SINGULAR (-6)     /* the requested system has no unique solution (see the solve) */

/* Basis along the non-periodic axis 0. */
#define SGM_SHEN_DIRICHLET 1  /* phi_l = T_l - T_{l+2}, l = 0..N-3 (eq. chebdirichlet)              */
#define SGM_SHEN_BIHARMONIC 2 /* phi_l = T_l - 2(l+2)/(l+3) T_{l+2} + (l+1)/(l+3) T_{l+4},
                                 l = 0..N-5 (eq. chebbiharmonic)                                    */
#define SGM_CHEBYSHEV 3       /* phi_l = T_l, l = 0..N-1 (regular Chebyshev basis, Sec. 3.1)        */
#define SGM_SHEN_NEUMANN 4    /* phi_l = T_l - (l/(l+2))^2 T_{l+2}, l = 0..N-3: Shen's Neumann basis
                                 (Sec. 3.1 names it without a formula; this is the standard one,
                                 phi_l'(+-1) = 0)                                                  */

/* Legendre-family bases (Sec. 3.1; Legendre-Gauss points and weights, Sec. 3.4.2):
 * the physical x axis then holds the N zeros of L_N in descending order, the
 * transforms along x are dense O(N^2) products (no fast algorithm exists), and
 * N <= 512. */
#define SGM_LEGENDRE 5        /* phi_l = L_l, l = 0..N-1                                           */
#define SGM_LEG_DIRICHLET 6   /* phi_l = L_l - L_{l+2}, l = 0..N-3 (eq. shen_legendre_basis)       */
#define SGM_LEG_NEUMANN 7     /* phi_l = L_l - l(l+1)/((l+2)(l+3)) L_{l+2}, l = 0..N-3 (phi' = 0
                                 at +-1; named in Sec. 3.1, formula the standard one)              */
#define SGM_LEG_BIHARMONIC 8  /* phi_l = L_l - 2(2l+5)/(2l+7) L_{l+2} + (2l+3)/(2l+7) L_{l+4},
                                 l = 0..N-5 (eq. legbiharmonic, read with l for k and the missing
                                 L_{l+4}; phi = phi' = 0 at +-1)                                   */

/* Transform kind of the last (contiguous) periodic axis. */
#define SGM_R2C 1 /* real physical data, M/2+1 coefficients (R2CBasis, Sec. 3.1)  */
#define SGM_C2C 2 /* complex physical data, M coefficients (C2CBasis, Sec. 3.1)   */

typedef struct sgm_plan_s* sgm_plan;

typedef struct {
    int ndim;      /* 2: [x][y]; 3: [x][y][z]                                          */
    int basis;     /* SGM_SHEN_DIRICHLET | SGM_SHEN_BIHARMONIC | SGM_CHEBYSHEV |
                      SGM_SHEN_NEUMANN | SGM_LEGENDRE | SGM_LEG_DIRICHLET |
                      SGM_LEG_NEUMANN | SGM_LEG_BIHARMONIC                             */
    int N;         /* points along x: >= 3 (Dirichlet, Neumann), >= 5 (biharmonic), >= 2 */
    int M1;        /* points along y, >= 1                                             */
    int M2;        /* points along z (ndim = 3), >= 1; ignored for ndim = 2            */
    int kind_last; /* SGM_R2C | SGM_C2C for the last axis (y if ndim = 2, z if 3)      */
    double Ly, Lz; /* periods of y and z; 0 means 2 pi.  Used only by the solves.      */
    int autotune;  /* 0: default kernels (register-resident FFTs for lengths 2^a 3^b with a
                      compiled instance, generic LDS kernels otherwise); 1: time the
                      candidates once at creation and keep the fastest (register
                      kernels per axis, rows per lane of the solves); 2: generic
                      LDS kernels only; 16 + v: pin register-kernel variant v
                      (0..7) wherever it is compiled (diagnostics) */
} sgm_plan_desc;

/* Create a plan for the tensor-product space V(x) x V^p(y) [x V^p(z)] (Sec. 4,
 * TensorProductSpace).  Uploads twiddle, recombination, projection and
 * solver tables and allocates one spectral-sized workspace on the current
 * device.  stream (a hipStream_t, null for the default stream) carries the
 * uploads and, with autotune = 1, the timing runs; the call synchronises that
 * stream before it returns, and leaves other streams alone.  Errors:
 * INVALID_ARG (null pointers, bad enums), UNSUPPORTED_SIZE (N below the basis
 * minimum, sizes above 65536 points per axis), OOM, HIP. */
sgm_status sgm_plan_create(const sgm_plan_desc* desc, void* stream, sgm_plan* out);
sgm_status sgm_plan_destroy(sgm_plan plan);

/* Physical and spectral shapes in elements (unused trailing dims are 1). */
sgm_status sgm_plan_shapes(sgm_plan plan, int64_t phys[3], int64_t spec[3]);

/* The N points of the x axis (the mesh along x, Sec. 3.4.2) into the HOST array
 * x[N]: Gauss-Chebyshev points cos((2j+1) pi / (2N)) for the Chebyshev family,
 * the Legendre-Gauss points (descending) for the Legendre family. */
sgm_status sgm_plan_points(sgm_plan plan, double* x);

/* Forward transform u -> u_hat (Sec. 4 and Sec. 3.4.2): Fourier transforms
 * with 1/M scaling along the periodic axes (last axis first), then the Shen
 * forward transform u_hat = B^{-1} S(u) along x (eq. projection), i.e. the
 * weighted L2 projection onto the basis.  u: physical (real for R2C,
 * complex for C2C); u_hat: spectral complex.  u and u_hat must not overlap;
 * u is not modified. */
sgm_status sgm_forward(sgm_plan plan, const void* u, void* u_hat, void* stream);

/* Backward transform u_hat -> u: u(x_j, y, z) = sum_l u_hat_l phi_l(x_j) e^{i(my+nz)}
 * (eq. fast_shen, eq. ufourier), unnormalised.  For R2C the imaginary parts of
 * the n = 0 and n = M/2 coefficients are ignored.  u_hat is not modified. */
sgm_status sgm_backward(sgm_plan plan, const void* u_hat, void* u, void* stream);

/* sgm_backward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and result, but the x pass writes its intermediate into a library-owned
 * static device array of 32 MiB (2^21 complex elements; one per device, held until
 * the process ends) instead of the plan's workspace.  The call itself allocates
 * nothing.  INVALID_ARG, before any device call, if the plan's spectral array has
 * more than 2^21 complex elements (e.g. 3D spaces above about 128^3).  Every call on
 * one device shares that array: calls that overlap on one device (any plan, any
 * stream) race.  u_hat is not modified. */
sgm_status sgm_backward_noalloc(sgm_plan plan, const void* u_hat, void* u, void* stream);

/* Scalar product f_tilde_l = (f, phi_l)^N_w after the Fourier transforms
 * (Sec. 4, right-hand side formula; the (2 pi)^(d-1) factor is dropped on both
 * sides of every solve).  Same layouts as sgm_forward. */
sgm_status sgm_scalar_product(sgm_plan plan, const void* f, void* f_tilde, void* stream);

/* Helmholtz solve alpha u - lap u = f for a Shen-Dirichlet plan, Chebyshev
 * (SGM_SHEN_DIRICHLET) or Legendre (SGM_LEG_DIRICHLET), or a Shen-Neumann plan
 * (SGM_SHEN_NEUMANN, SGM_LEG_NEUMANN: homogeneous Neumann conditions u'(+-1) = 0);
 * other bases are rejected: per Fourier wavenumber column with
 * kappa^2 = (2pi m/Ly)^2 + (2pi n/Lz)^2, solves
 * (-A + (kappa^2 + alpha) B) u_hat = f_tilde (eq. cheb_poisson, eq. laplace),
 * A_ml = (phi_l'', phi_m), B_ml = (phi_l, phi_m) in the basis's own weighted inner
 * product (Chebyshev weight, resp. weight 1: then -A = diag(4l + 6) and B has
 * 2/(2l+1) + 2/(2l+5) on the diagonal and -2/(2l+5) two places off it).  Neumann:
 * with r_l = (l/(l+2))^2, -A_ll = 2 pi l^2 (l+1)/(l+2), -A_ml = pi (1 - r_m) l^2
 * for l >= m + 2 of the same parity, B_ll = (pi/2)(c_l + r_l^2), B_{l,l+2} =
 * -(pi/2) r_l; Legendre-Neumann: with s_l = l(l+1)/((l+2)(l+3)), -A = diag((4l + 6)
 * s_l), B_ll = 2/(2l+1) + s_l^2 2/(2l+5), B_{l,l+2} = -s_l 2/(2l+5).  Neumann bases:
 * alpha = 0 returns SGM_ERR_SINGULAR before any device work (the constant mode of
 * the zero wavenumber is then undetermined).
 * f_tilde and u_hat are spectral arrays (rows >= N-2 of f_tilde ignored); they
 * may be the same pointer (in-place).  alpha >= 0.  INVALID_ARG otherwise.  The
 * first call with a given alpha also refreshes a plan-owned table of elimination
 * states at chain-segment boundaries (one extra kernel on the same stream); calls
 * that overlap on one plan race. */
sgm_status sgm_helmholtz_solve(sgm_plan plan, double alpha, const void* f_tilde, void* u_hat, void* stream);

/* The same solve from the physical right-hand side: u_hat = solve(alpha,
 * scalar_product(f)), i.e. sgm_scalar_product followed by sgm_helmholtz_solve
 * (Sec. 4: right-hand side scalar product, then the per-wavenumber solve).  f:
 * physical real array (as u in sgm_forward), u_hat: spectral output; they must
 * not overlap; f is not modified.  Where the plan allows (Chebyshev x axis of 256
 * points on 8-column tiles) the Chebyshev pass and the solve run as one kernel, the
 * solve reading the scalar product from on-chip memory; otherwise the two
 * calls run in turn.  Table refresh and races as sgm_helmholtz_solve. */
sgm_status sgm_helmholtz_solve_physical(sgm_plan plan, double alpha, const void* f, void* u_hat, void* stream);

/* Biharmonic solve lap^2 u = f for a Shen-biharmonic plan, Chebyshev
 * (SGM_SHEN_BIHARMONIC) or Legendre (SGM_LEG_BIHARMONIC) (Sec. 4): per column
 * (S - 2 kappa^2 A + kappa^4 B) u_hat = f_tilde with S_ml = (phi_l'''', phi_m) in the
 * basis's weighted inner product (Legendre: S = diag(2 (2l+3)^2 (2l+5)), A and B
 * banded).  Same layout, aliasing rules and first-call table fill as
 * sgm_helmholtz_solve; other bases are rejected (INVALID_ARG). */
sgm_status sgm_biharmonic_solve(sgm_plan plan, const void* f_tilde, void* u_hat, void* stream);

/* Derivative and projection (Sec. 5: the Dx operator, nested for mixed
 * derivatives, and project(Dx(u, ...), W0, uh_hat=u_hat)).  u_hat holds the
 * coefficients of u in `plan`'s space; du_hat receives the coefficients, in the
 * space of `target`, of the weighted L2 projection of
 * d^(ox+oy+oz) u / dx^ox dy^oy dz^oz, order = {ox, oy, oz} (y the middle and z the
 * last axis for ndim = 3, y the last axis for ndim = 2, where oz must be 0; each
 * 0..8).  For a Chebyshev-family plan target->basis is SGM_CHEBYSHEV, where the
 * result is the derivative's Chebyshev coefficients exactly (it is a polynomial of
 * degree < N), SGM_SHEN_DIRICHLET, the projection the paper uses when the
 * derivative vanishes at x = +-1 (exact then, a least-squares fit otherwise), or
 * SGM_SHEN_NEUMANN; for a Legendre-family plan (every Legendre basis may be the
 * source) it is SGM_LEGENDRE, SGM_LEG_DIRICHLET or SGM_LEG_NEUMANN, the same
 * projections in the Legendre inner product (weight 1).  Other targets, and a
 * target of the other family, are rejected (INVALID_ARG).  target must have the
 * same ndim, N, M1, M2, kind_last and periods.  Along a periodic axis of M points
 * coefficient k is multiplied by (2 pi i k / L)^o; for even M the odd derivatives
 * of the Nyquist coefficient are zero.  Spectral layouts as in sgm_forward; u_hat
 * and du_hat must not overlap.  UNSUPPORTED_SIZE for N > 512. */
sgm_status sgm_project_derivative(sgm_plan plan, sgm_plan target, const int order[3], const void* u_hat,
                                  void* du_hat, void* stream);

/* Small 2D spaces (ndim = 2, N <= 64, M1 <= 64, not biharmonic) with autotune 0 or 1
 * run every forward / backward / scalar-product call as one kernel (dense products in
 * one work-group's LDS); their pass timing then records the whole call as the x pass
 * (kind 4, 5 or 6).
 * Per-pass timing (diagnostics).  enable = 0: off; 1: every pass kernel this plan
 * launches is bracketed by two hipEvents recorded on the caller's stream (the
 * events are created on first use and owned by the plan); SGM_TIMING_ONLY | bits:
 * only the pass kinds whose bit (1 << kind) is set.  Pass kinds:
 * 0 last-axis forward FFT, 1 last-axis backward FFT, 2 middle-axis forward FFT,
 * 3 middle-axis backward FFT, 4 Chebyshev forward (projection), 5 Chebyshev
 * scalar product, 6 Chebyshev backward, 7 Galerkin solve.
 * sgm_plan_pass_times waits for the recorded events, adds their durations to
 * ms[SGM_NPASS] and launch counts to count[SGM_NPASS] (running totals since the
 * last reset) and, if reset != 0, clears the totals afterwards. */
#define SGM_NPASS 8
#define SGM_TIMING_ONLY 0x100
sgm_status sgm_plan_timing(sgm_plan plan, int enable);
/* Register-kernel variant in use per axis (x, y, z): 0..7, or -1 where the axis runs
 * the generic LDS kernels (diagnostics; chosen at creation, see autotune). */
sgm_status sgm_plan_variants(sgm_plan plan, int variant[3]);
/* Layout of the plan's Galerkin solves (diagnostics): each (column, parity) chain is
 * split over `lanes` lanes of a wave with `rows` rows each (16 by default; plans
 * created with autotune = 1 time 16 and 8 rows per lane and keep the faster);
 * lanes = rows = 0 where the solves run one chain per lane or the basis has none. */
sgm_status sgm_plan_solve_layout(sgm_plan plan, int* lanes, int* rows);
/* Set the rows per lane (8 or 16) of the plan's segmented solves: re-sizes the
 * boundary table (a device synchronisation, then a new allocation owned by the plan).
 * INVALID_ARG for other values, for plans without segmented solves and where the
 * chains would need more than 16 lanes. */
sgm_status sgm_plan_set_solve_rows(sgm_plan plan, int rows);
sgm_status sgm_plan_pass_times(sgm_plan plan, double ms[SGM_NPASS], int64_t count[SGM_NPASS], int reset);

/* ---- Complex Ginzburg-Landau, ragged batch (Sec. 6) ------------------------------
 * u_t = u + (1 + i b) lap u - (1 + i c)|u|^2 u on the periodic square [-L/2, L/2)^2
 * with Fourier x Fourier bases (eq. Ginz_var; the paper's case is b = 0, c = 1.5,
 * L = 100).  A batch holds `count` independent problems of possibly different
 * sizes N_i; every packed array stores problem i as an N_i x N_i C-ordered
 * complex array ([x][y], FFT order for spectra) at complex offset offsets[i].
 * The nonlinear term uses the 3/2 rule: retained modes evaluated on the
 * floor(3N/2)^2 grid (other padded modes zero), product formed there, forward
 * transformed with 1/M per axis and truncated (Sec. 6, padded transforms). */
#define SGM_RK4 1   /* the explicit four-stage Runge-Kutta scheme of Sec. 6            */
#define SGM_IFRK4 2 /* the same RK4 after the integrating factor exp(-Lhat t), Lhat =
                       1 - (1 + i b)|k|^2 (Lawson); exact for the linear part          */

typedef struct sgm_gl_s* sgm_gl;

typedef struct {
    int count;      /* number of problems, >= 1                                          */
    const int* N;   /* host array[count]: points per side, 2 <= N_i <= 4096              */
    double L;       /* side of the square (> 0)                                          */
    double b, c;    /* equation coefficients                                             */
    double dt;      /* time step of sgm_gl_step                                          */
    int scheme;     /* SGM_RK4 | SGM_IFRK4                                               */
    int graph;      /* 1: sgm_gl_step captures one step as a hipGraph (per state pointer
                       and stream) and replays it; 0: launches the kernels directly      */
    int tune;       /* launch configuration of the time-stepping kernels: 0 default;
                       1 time every candidate on one step at creation (on the current
                       device, on the creation stream) and keep the fastest; 16 + k pin
                       candidate k, 0 <= k < SGM_GL_NVARIANT                             */
} sgm_gl_desc;
#define SGM_GL_NVARIANT 6 /* candidate = 2 * geometry (3 FFT tilings) + grid mode
                             (0 persistent grid, 1 one work-group per work item)         */

/* Create a batch: uploads the per-problem descriptors, work lists and twiddle
 * tables and allocates two state-sized stage buffers and one padded workspace
 * (sum_i N_i floor(3 N_i / 2) complex elements).  stream (hipStream_t, null for
 * the default stream) carries the uploads and, with tune = 1, the timing runs;
 * the call synchronises that stream before it returns.  Errors: INVALID_ARG,
 * UNSUPPORTED_SIZE, OOM, HIP. */
sgm_status sgm_gl_create(const sgm_gl_desc* desc, void* stream, sgm_gl* out);
sgm_status sgm_gl_destroy(sgm_gl gl);
/* Number of problems of the batch. */
sgm_status sgm_gl_count(sgm_gl gl, int* count);
/* Launch configuration in use (0 <= *variant < SGM_GL_NVARIANT). */
sgm_status sgm_gl_variant(sgm_gl gl, int* variant);
/* offsets[0..count]: packed layout (complex elements); offsets[count] = total. */
sgm_status sgm_gl_offsets(sgm_gl gl, int64_t* offsets);
/* u_hat = (1/N^2) sum_x u(x) e^{-i k.x} per problem (Sec. 3.4.1 forward, both axes). */
sgm_status sgm_gl_forward(sgm_gl gl, const void* u, void* u_hat, void* stream);
/* u(x) = sum_k u_hat_k e^{i k.x} per problem (unnormalised). */
sgm_status sgm_gl_backward(sgm_gl gl, const void* u_hat, void* u, void* stream);
/* rhs = (1 - (1 + i b)|k|^2) u_hat - F_trunc[(1 + i c)|u_p|^2 u_p] with k = (2 pi/L) *
 * integer wavenumbers (the right-hand side of eq. Ginz_var after dividing by the
 * diagonal mass (2 pi)^2).  u_hat and rhs must not overlap. */
sgm_status sgm_gl_rhs(sgm_gl gl, const void* u_hat, void* rhs, void* stream);
/* Advance every problem by nsteps steps of dt in place (nsteps >= 0).  Calls that
 * overlap on one batch object race (they share its stage buffers). */
sgm_status sgm_gl_step(sgm_gl gl, void* u_hat, int nsteps, void* stream);

/* ---- FNO-style surrogate for Ginzburg-Landau states --------------------------------
 * Learned map u(t) -> u(t + s dt) on an H x W periodic grid, the complex state split
 * into two real channels: x is fp32 channels-last [B][H][W][2] (Re, Im).
 *   a = x W_l + b_l (lift to `width` channels); `layers` times:
 *   z = IDFT_K(R_l DFT_K(a)) + a W_p + b_p, a = gelu(z) (no gelu after the last);
 *   out = gelu(a W_1 + b_1) W_2 + b_2;  pred = x + out.
 * DFT_K keeps ky in {0..K-1, H-K..H-1}, kx in {0..K-1} (1/(HW) normalised); IDFT_K
 * is the real inverse of that half spectrum (weight 2 for kx > 0).  Activations
 * and GEMM operands are bfloat16 on the matrix cores with fp32 accumulation;
 * parameters, gradients and Adam moments are fp32.  Loss: mean over samples of
 * ||pred - target||_2 / ||target||_2.
 * Flat parameter order: W_l[2][C], b_l[C], per layer {R_re[2K][K][C][C],
 * R_im[2K][K][C][C], W_p[C][C], b_p[C]}, W_1[C][P], b_1[P], W_2[P][2], b_2[2]. */
typedef struct sgm_fno_s* sgm_fno;

typedef struct {
    int H, W;       /* grid; 2 * modes <= H, W                                   */
    int width;      /* channels C                                                */
    int modes;      /* retained modes K per direction                            */
    int layers;     /* spectral layers                                           */
    int hidden;     /* projection width P                                        */
    int max_batch;  /* largest batch any call will use (sizes the workspace)     */
} sgm_fno_desc;

/* Allocate parameters (seeded initialisation), Adam state and a workspace for
 * max_batch samples (about (2 layers + 3) B H W C bf16 plus B H W P).
 * SGM_ERR_INVALID_ARG, before any device call, for sizes out of range or
 * max_batch * 4 * modes^2 * width >= 2^31 (the spectral buffers' element count). */
sgm_status sgm_fno_create(const sgm_fno_desc* desc, uint64_t seed, sgm_fno* out);
sgm_status sgm_fno_destroy(sgm_fno f);
sgm_status sgm_fno_num_params(sgm_fno f, int64_t* n);
/* Host copies of the flat fp32 parameter vector (set also resets Adam). */
sgm_status sgm_fno_set_params(sgm_fno f, const float* host);
sgm_status sgm_fno_get_params(sgm_fno f, float* host);
/* pred = net(x) for `batch` samples (device arrays [batch][H][W][2]); with an
 * ensemble set (sgm_fno_set_ensemble) the average of its members.  With more than
 * one member pred must not overlap x. */
sgm_status sgm_fno_infer(sgm_fno f, const float* x, float* pred, int batch, void* stream);
/* Inference averaged over reflections of the periodic square (not in the paper;
 * the GL equation of Sec. 6, u_t = u + (1 + i b) lap u - (1 + i c)|u|^2 u on a
 * doubly periodic square, commutes with them, and so does its solution map):
 * pred = (1/m) sum_R R^{-1} net(R x) over m = `members` reflections R of the
 * H x W grid, (R u)[i][j] = u[s(i, j)]: 1 = the network alone, 4 = the identity and
 * the flips of rows (i -> H-1-i), of columns (j -> W-1-j) and of both, 2 = the
 * identity and the transpose, 8 = all eight (flips, then transpose).  Transposes
 * need H = W (else INVALID_ARG); other member counts are INVALID_ARG.  The first
 * call with members > 1 allocates two B_max x H x W x 2 float buffers, owned by
 * the network; inference then runs the network `members` times.  Applies to
 * sgm_fno_infer and to sgm_fno_advance_checked; training is unaffected. */
sgm_status sgm_fno_set_ensemble(sgm_fno f, int members);
/* Forward + loss + backward without an update: gradients to grads_host (num_params
 * floats, may be NULL) and the mean relative L2 loss to loss_host (may be NULL).
 * Synchronises the stream. */
sgm_status sgm_fno_grads(sgm_fno f, const float* x, const float* target, int batch, float* grads_host,
                         float* loss_host, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate lr; the batch
 * loss before the update goes to loss_host if it is not NULL (then synchronises). */
sgm_status sgm_fno_train_step(sgm_fno f, const float* x, const float* target, int batch, float lr,
                              float* loss_host, void* stream);
/* Per-sample relative L2 ||pred - target|| / ||target|| into rel_dev (device floats). */
sgm_status sgm_fno_rel_l2(sgm_fno f, const float* pred, const float* target, int batch, float* rel_dev,
                          void* stream);
/* Checkpoint: parameters and Adam state (binary file). */
sgm_status sgm_fno_save(sgm_fno f, const char* path);
sgm_status sgm_fno_load(sgm_fno f, const char* path);
/* n complex128 values <-> n (Re, Im) fp32 pairs (GL states to FNO inputs and back). */
sgm_status sgm_fno_pack(const void* u_c128, float* x, int64_t n, void* stream);
sgm_status sgm_fno_unpack(const float* x, void* u_c128, int64_t n, void* stream);

/* Surrogate advance with FP64 fallback.  `gl` holds B problems, all H x W (= the
 * FNO grid); u_hat is its packed spectral state, advanced in place by nsur
 * macro-steps of the surrogate, each standing for steps_per solver steps of gl's dt
 * (the network must have been trained for that stride).  Per macro-step a seeded
 * subset of NC = `gl_check`->count samples (evenly spaced, random offset; 1 <= NC <= B)
 * is also advanced by the FP64 solver `gl_check` (same N, L, b, c, dt) and judges the
 * surrogate by the relative L2 error ||pred - solver|| / ||solver|| of the physical
 * fields.  Acceptance, per macro-step:
 *   - more than max_fail_frac * NC checked samples above tol: the checks are taken as
 *     evidence that the unchecked samples fail too, and the FP64 solver `gl` advances
 *     the whole batch from the macro-step's starting state (the surrogate's prediction
 *     is discarded); max_fail_frac = 0 re-advances on any failed check;
 *   - otherwise every sample takes the surrogate's prediction except the failed
 *     checked ones, which take the checking solver's result.
 * max_fail_frac in [0, 1], else INVALID_ARG.  stats (may be NULL) accumulates into
 * the caller's struct (zero it before the first call).  The workspace (about
 * B H W 32 + NC H W 48 bytes) is allocated on the first call and re-allocated,
 * after a device synchronisation, whenever a call needs more.  The FP64 checks run
 * on a private second stream of the library (default priority), created on the
 * first call and overlapped with the inference; they are joined to `stream` before
 * the comparison.  Synchronises the stream once per macro-step. */
typedef struct {
    int n_checked;        /* samples checked by the solver                              */
    int n_fallback;       /* checked samples above tol                                  */
    float max_rel_l2;     /* largest checked relative L2 error                          */
    float mean_rel_l2;    /* mean checked relative L2 error                             */
    int n_batch_fallback; /* macro-steps in which the FP64 solver advanced every sample */
    int n_replaced;       /* samples whose new state came from an FP64 solver           */
} sgm_fno_stats;
sgm_status sgm_fno_advance_checked(sgm_fno f, sgm_gl gl, sgm_gl gl_check, void* u_hat, int nsur, int steps_per,
                                   double tol, double max_fail_frac, uint64_t seed, sgm_fno_stats* stats,
                                   void* stream);

/* ---- Autotuner memory ----------------------------------------------------------------
 * Plans created with autotune = 1 and GL batches created with tune = 1 time their
 * candidate kernels once per geometry (plan: device, ndim, basis, N, M1, M2, kind_last;
 * batch: device, scheme, sizes) and remember the choice in the process and in a
 * text file: $SGM_TUNE_CACHE if set ("off": no file), else
 * $XDG_CACHE_HOME/libsgm/tune.txt, else $HOME/.cache/libsgm/tune.txt.  A stored
 * choice is reused only if it names kernels this build compiled.  The file is
 * read and appended without locking (the last line for a key wins).
 * sgm_autotune_forget clears the in-process memory (the file is kept), so the next
 * tuned plan or batch reads the file or times again; sgm_autotune_cache_path copies
 * the file path (empty if none) into buf[len]. */
sgm_status sgm_autotune_forget(void);
sgm_status sgm_autotune_cache_path(char* buf, int len);

const char* sgm_status_string(sgm_status s);
const char* sgm_last_error(void);
int sgm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SGM_H */
