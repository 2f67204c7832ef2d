/*
 * pdf.h - C ABI of the MI355X (gfx950) Physics-Driven Fourier-Spectral (PDF)
 * inverse-scattering hot path.
 *
 * The library evaluates, for B independent data sets that share one
 * measurement geometry, the composite PDF loss (Sec. 3.2, Eqs. 13-19) of
 * truncated Fourier coefficients alpha of the induced currents (Sec. 2.3,
 * Eq. 9) and its gradient, applies Adam (Sec. 3.3), computes the
 * back-propagation start (Sec. 3.1) or the full CSI start, the CIE contrast
 * and the contrast-compensated image (Sec. 2.4, Eqs. 10-11), runs the
 * solver's coefficient network (Sec. 3.1, Fig. 4: Adam on network weights
 * instead of on alpha), and synthesises measured fields with an FP64
 * method-of-moments solve (Sec. 2.1, Eqs. 3-4).
 *
 * Conventions (all entry points)
 *   - Every function returns an int status: PDF_OK (0) or a negative code.
 *     No C++ exception crosses the ABI.  pdf_last_error(h) gives a message.
 *   - Complex arrays are interleaved (re, im), C-contiguous, in the
 *     handle's precision: float pairs for PDF_FP32, double pairs for PDF_FP64.
 *   - "_dev" pointers are device pointers owned by the caller; the handle
 *     owns its operator tables and scratch and frees them in pdf_destroy.
 *   - Calls are asynchronous on the stream given to pdf_setup unless stated.
 *     One handle is used from one host thread / stream at a time.
 *   - Grid: row i runs along y, column j along x, pixel n = i*M + j, pixel
 *     centres at centre - side/2 + (index + 1/2) * side / M.
 *   - Fourier coefficients alpha: [B][Ni][K][K], ky outer, kx inner, both
 *     k = -floor(K/2) ... ceil(K/2)-1.  Odd K is a centred set; even K = 2 M_F
 *     is the paper's set of four M_F x M_F corner blocks (Sec. 2.3).
 *     J[i][j] = sum alpha[ky][kx] exp(+2 pi i (ky i + kx j) / M).
 *   - Time dependence exp(-i w t); Green's function (i/4) H0^(1)(k0 r).
 */
#ifndef PDF_H
#define PDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PDF_OK = 0,
  PDF_EINVAL = -1,       /* bad argument (null pointer, size out of range)        */
  PDF_ENOMEM = -2,       /* device or host allocation failed                      */
  PDF_EHIP = -3,         /* a HIP runtime call or kernel launch failed            */
  PDF_ENONFINITE = -4,   /* non-finite loss, zero data norm or zero E_inc norm    */
  PDF_EUNSUPPORTED = -5  /* valid request this build does not implement           */
};

enum { PDF_FP32 = 0, PDF_FP64 = 1 };

#define PDF_PARAMS_VERSION 2
#define PDF_LOSS_STRIDE 8   /* doubles per instance in a loss buffer */

/* Loss buffer layout, per instance: [State, Data, Bound, TV, Bridge, Total,
   max |R| (diagnostic), non-finite flag (1.0 if any term is not finite)]. */

typedef struct pdf_handle pdf_handle;

typedef struct {
  int32_t M;        /* pixels per side of the inversion grid                  */
  double side;      /* side length of the square domain, metres               */
  double cx, cy;    /* domain centre, metres                                  */
} pdf_grid;

typedef struct {
  int32_t n;        /* number of antennas                                     */
  const double* xy; /* host [n][2] (x, y) positions, metres                   */
} pdf_array;

typedef struct {
  int32_t version;     /* PDF_PARAMS_VERSION                                          */
  int32_t precision;   /* PDF_FP32 or PDF_FP64 arithmetic for the whole path          */
  double beta;         /* CIE contraction parameter (Sec. 2.2, Eq. 6); paper: 6       */
  double lam_bound;    /* weight of L^Bound (Eq. 17); paper: 1e-3                     */
  double lam_tv;       /* weight of L^TV (Eq. 18); paper: 1e-5                        */
  double lam_bridge;   /* weight of L^Bridge (Eq. 19); paper: 1e-5                    */
  double tau_b;        /* bridge threshold (Eq. 19); paper: 0.5                       */
  double eps_tv;       /* added under the TV square root; 1e-12                       */
  double eps_abs;      /* |chi| smoothing in L^Bridge, sqrt(|chi|^2 + eps_abs); 1e-12 */
  double cco_tau;      /* CCO threshold tau (Eq. 11); paper: 3                         */
  double cco_eta_max;  /* CCO maximum gain (Eq. 11); paper: 0.1                        */
  double cco_delta;    /* CCO slope delta (Eq. 11); paper: 0.5                         */
  int32_t gf_radius;   /* self-guided filter box radius; 1                             */
  double gf_eps;       /* self-guided filter regulariser; 1e-2                         */
  double lr;           /* Adam learning rate (Sec. 3.3); paper: 1e-2                  */
  double adam_b1, adam_b2, adam_eps;   /* 0.9, 0.999, 1e-8                             */
  int32_t r_stopgrad;  /* 1: treat R as a constant in the gradient                     */
  /* Added in version 2 (a version-1 struct ends before it and reads as 0). */
  int32_t cco_in_loss; /* 1: evaluate the chi-dependent loss terms on chi_CCO (Sec. 2.4,
                          Eqs. 10-11) instead of chi: the regularisers (Eqs. 17-19) on
                          chi_CCO and the state residual (Eq. 15) with R_c = beta chi_CCO /
                          (1 + beta chi_CCO), the gradient taken through the CCO.  The paper
                          applies the CCO after the iterations only (0, the default).
                          Single-frequency handles on grids up to 64 x 64 (96 x 96 in FP32);
                          PDF_EUNSUPPORTED otherwise.                                  */
} pdf_params;

/* Fill *p with the paper's defaults (precision PDF_FP32).  Host only. */
int pdf_default_params(pdf_params* p);

/* Build operator tables for one geometry (Sec. 2.1, Eqs. 3-4) and scratch for
 * `batch` data sets.  FP64 on the host: Hankel-function tables of the domain
 * operator G_D (circular-cell method of moments), its spectrum on the 2M x 2M
 * circulant embedding, the receiver operator G_S [Ns][N] and the incident
 * fields [Ni][N] (unit magnitude at the domain centre); then cast to the
 * handle's precision and copied to the device.  Synchronous.
 *   grid, tx, rx, params: host structs (params may be NULL for defaults).
 *   freq_hz: frequency.  K: truncation per axis, 1 <= K <= M.
 *   stream: hipStream_t for every later call (must not be NULL).
 * Supported: M in {8, 16, 32, 48, 64, 96, 128, 256}; Ni, Ns >= 1 (FP32: at most
 * 64 each).  Grids whose padded half tile does not fit one CU's LDS (FP32 from
 * 128, FP64 from 96) run the convolution in passes through a device array of
 * B Ni M 2M complex values that the handle allocates.
 * Errors: PDF_EINVAL (bad sizes / null), PDF_EUNSUPPORTED (other M),
 * PDF_ENOMEM, PDF_EHIP, PDF_ENONFINITE (||E_inc|| = 0). */
int pdf_setup(const pdf_grid* grid, double freq_hz, const pdf_array* tx,
              const pdf_array* rx, int32_t K, int32_t batch,
              const pdf_params* params, void* stream, pdf_handle** out);

/* Frequencies of a multi-frequency reconstruction. */
typedef struct {
  int32_t n_freq;    /* 1 .. 8                                                  */
  const double* hz;  /* host [n_freq] frequencies, Hz                           */
} pdf_freq;

/* pdf_setup for data measured at several frequencies.  The medium is taken as
 * non-dispersive: one contrast chi (and so one R of Eq. 7) for all
 * frequencies, while the coefficients, currents, fields and operators are per
 * frequency.  R is the per-pixel least-squares solution over all frequencies
 * and incidences with each frequency weighted by 1 / ||E_inc,f||^2 (so that R
 * minimises the summed state loss); L^State and L^Data (Eqs. 15-16) are
 * summed over the frequencies, each normalised by its own ||E_inc,f||^2 and
 * ||E_sca,f||^2; the regularisers act on the one chi.  With n_freq == 1 this
 * is pdf_setup.  With n_freq > 1 the handle holds one reconstruction
 * (batch must be 1, else PDF_EUNSUPPORTED) and every per-instance array
 * carries the frequencies outermost: alpha, gradient [F][Ni][K][K]; Adam
 * moments [F][Ni][K][K][2]; measured fields [F][Ni][Ns]; loss [1][8]; step
 * counter [1]; images [1][M][M].  Such a handle serves pdf_set_data,
 * pdf_loss_grad, pdf_step, pdf_init_alpha (the back-propagation start with the
 * joint contrast and one exact line-search step on the summed L^CSI),
 * pdf_image, pdf_reconstruct, pdf_autotune and pdf_set_tiles; the other
 * entry points return PDF_EUNSUPPORTED for it.  Other arguments and errors as
 * pdf_setup. */
int pdf_setup_freq(const pdf_grid* grid, const pdf_freq* freq, const pdf_array* tx,
                   const pdf_array* rx, int32_t K, int32_t batch,
                   const pdf_params* params, void* stream, pdf_handle** out);

/* Host-only FP64 operator tables (no device work), for checking pdf_setup:
 * ghat [2M][2M] (FFT of the embedded G_D kernel, unscaled), gs [Ns][N],
 * einc [Ni][N], all complex128 host buffers allocated by the caller.
 * Any output pointer may be NULL to skip it. */
int pdf_tables_host(const pdf_grid* grid, double freq_hz, const pdf_array* tx,
                    const pdf_array* rx, double* ghat, double* gs, double* einc);

/* Copy measured fields E_sca [B][Ni][Ns] (device, handle precision) into the
 * handle and compute each instance's ||E_sca||^2.  Errors: PDF_EINVAL. */
int pdf_set_data(pdf_handle* h, const void* esca_dev);

/* Loss and gradient at alpha (Sec. 3.2, Eqs. 13-19; the adjoint is the chain
 * rule through every step, with the per-pixel least-squares contrast
 * R = beta sum J conj(E) / sum |E|^2 (Eqs. 6-7)).
 *   alpha_dev: [B][Ni][K][K] complex.  grad_dev: same shape, may be NULL
 *   (then only the forward kernels and the loss pass run, no adjoint).
 *   loss_dev: device double [B][PDF_LOSS_STRIDE], may be NULL.
 * Gradient convention: dL/dRe + i dL/dIm (that of PyTorch). */
int pdf_loss_grad(pdf_handle* h, const void* alpha_dev, void* grad_dev, double* loss_dev);

/* One Adam step (Sec. 3.3) on alpha in place: loss and gradient at alpha,
 * then the bias-corrected update of (Re, Im) pairs.
 *   m_dev, v_dev: [B][Ni][K][K][2] real moment buffers (zero before step 1).
 *   t_dev: device int32 [B], steps already taken per instance; incremented.
 *   loss_dev: as in pdf_loss_grad (loss before the update), may be NULL.
 * Graph-capturable: all step-dependent state is in device memory. */
int pdf_step(pdf_handle* h, void* alpha_dev, void* m_dev, void* v_dev,
             int32_t* t_dev, double* loss_dev);

/* Size of the library's static device scratch (one copy per device, held from
 * the first pdf_setup on that device until the process ends). */
#define PDF_STATIC_SCRATCH_BYTES (32u << 20)

/* pdf_init_alpha_csi for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation with the same kernels and bitwise the same
 * result, but its conjugate-gradient workspace (B Ni K^2 complex values plus
 * two doubles per instance, each part rounded up to 256 bytes) lives in the
 * library's static scratch instead of a buffer the handle allocates.  The call
 * allocates and frees nothing.
 *   Errors: PDF_EINVAL if n_iter > 1 and the workspace exceeds
 *   PDF_STATIC_SCRATCH_BYTES (e.g. FP32, B = 256, Ni = 32, K = 15 needs
 *   14.75 MB and fits); PDF_EHIP if the scratch's address could not be found
 *   on the handle's device at pdf_setup.
 * Every call on one device shares that device's scratch and leaves its
 * contents behind (nothing in it needs to start at zero: each value is
 * written before it is read within a call), so calls that overlap on one
 * device race: run them on one stream, or order their streams. */
int pdf_init_alpha_csi_noalloc(pdf_handle* h, int32_t n_iter, void* alpha_dev);

/* Start value alpha_0 (Sec. 3.1): back-propagation image, R_0 by Eq. 7, and
 * one gradient step on L^CSI (Eq. 12) from zero with the exact line-search
 * step size.  alpha_dev: output [B][Ni][K][K]. */
int pdf_init_alpha(pdf_handle* h, void* alpha_dev);

/* The full CSI start (Sec. 3.1), which the paper sets aside for its cost:
 * L^CSI (Eq. 12) with R fixed at the back-propagation R_0 is quadratic in
 * alpha, and n_iter >= 1 conjugate-gradient steps from zero minimise it
 * (directions p_1 = -g_1, p_k = -g_k + (|g_k|^2 / |g_{k-1}|^2) p_{k-1}, each
 * with its exact step).  n_iter = 1 gives pdf_init_alpha's start.  Each
 * further step costs about two loss evaluations.  alpha_dev: output
 * [B][Ni][K][K].  The library keeps a workspace of B Ni K^2 complex values in
 * the handle (allocated on the first call with n_iter > 1). */
int pdf_init_alpha_csi(pdf_handle* h, int32_t n_iter, void* alpha_dev);

/* Images at alpha: chi = R/(beta(1-R)) and the CCO image (Eqs. 10-11).
 *   chi_dev, chi_cco_dev: [B][M][M] complex outputs, either may be NULL.
 *   eps_true_dev: [B][M][M] complex relative permittivity, may be NULL.
 *   err_dev: device double [B]: ||(1+chi_cco) - eps|| / ||eps||, may be NULL
 *   (requires eps_true_dev). */
int pdf_image(pdf_handle* h, const void* alpha_dev, void* chi_dev, void* chi_cco_dev,
              const void* eps_true_dev, double* err_dev);

typedef struct {
  int32_t iters_run;       /* Adam steps taken by the slowest instance            */
  int32_t n_reached;       /* instances whose image error reached its target       */
  double seconds;          /* wall time of the call                                */
} pdf_report;

/* A full reconstruction of every instance (Sec. 3, Fig. 3): alpha_0 (or the
 * caller's start), up to n_iter Adam steps replayed from a captured HIP graph
 * of n_check steps, then the CCO image.  With eps_true_dev, the image error
 * ||(1 + chi_cco) - eps|| / ||eps|| is evaluated at the start and every
 * n_check steps; with target_err_dev an instance stops updating once its
 * error is <= its target, and the call returns when all have stopped.
 * Synchronous.
 *   alpha_dev: [B][Ni][K][K] in/out (in: start if start_given != 0).
 *   eps_true_dev: [B][M][M] complex, may be NULL (no error checks).
 *   target_err_dev: device double [B], may be NULL (no early stop).
 *   reached_iter_dev: device int32 [B] out, step at which the target was met
 *     (-1 if never), may be NULL.
 *   best_err_dev / best_iter_dev: device double / int32 [B] out, lowest
 *     checked error and its step, may be NULL.
 *   chi_cco_dev: [B][M][M] output, may be NULL. */
int pdf_reconstruct(pdf_handle* h, int32_t n_iter, int32_t n_check, int32_t start_given,
                    void* alpha_dev, const void* eps_true_dev, const double* target_err_dev,
                    int32_t* reached_iter_dev, double* best_err_dev, int32_t* best_iter_dev,
                    void* chi_cco_dev, pdf_report* rep);

/* Tile shapes and FFT plans of this handle's FP32 kernels, chosen by timing
 * `reps` launches of each candidate on the handle's own buffers: the G_S^H
 * GEMM's column tiles per wavefront (1, 2 or 4 tiles of 32 pixels), the
 * pixel reduction's load batch (4 incidences at four wavefronts per SIMD, or
 * 8 at two), and for each convolution kernel its plan: 0 keeps only the M
 * stored rows of the padded tile in LDS with in-place row passes (two
 * barriers each; at M = 64 two workgroups per CU), 1 keeps all 2M rows and
 * alternates the row passes between the halves (one barrier each, twice the
 * LDS; grids where that exceeds one CU's LDS, M = 96, have plan 0 only and
 * run it whatever is set).  The plans are timed as pairs inside whole
 * loss-gradient passes.
 * Every candidate computes each result in the same order, so the choice
 * changes timing only, never a value.  choice: host int32 [4] out (column
 * tiles, load batch, forward plan, adjoint plan), may be NULL; ms: host
 * double [9] out (three GEMM and two reduction timings, then the
 * loss-gradient pass with plans (0,0), (0,1), (1,0), (1,1)), may be NULL.
 * FP64 handles and grids with M*M not a multiple of 32 keep the defaults
 * (2, 4, 0, 0).  Synchronous; overwrites the handle's scratch arrays and its
 * internal Adam moments (every pdf_reconstruct re-initialises them), not
 * alpha or the data. */
int pdf_autotune(pdf_handle* h, int32_t reps, int32_t* choice, double* ms);
/* Sets the choices directly (ct in {1, 2, 4}, pb in {4, 8}, plans 0 or 1). */
int pdf_set_tiles(pdf_handle* h, int32_t ct, int32_t pb, int32_t fwd_pp, int32_t adj_pp);

/* Uneven batching: the reconstructions of n handles (different grids, antenna
 * counts, truncations, batch sizes and precisions) advanced together.  Every
 * n_check steps of all still-running handles are one HIP graph made of one
 * branch per handle (that handle's kernels, specialised for its shape) with no
 * dependencies between branches, so the handles run concurrently on the GPU;
 * the graph is rebuilt only when a handle stops.  Array arguments hold n
 * entries with pdf_reconstruct's meaning for hs[i] (an array may be NULL
 * where pdf_reconstruct allows NULL, meaning NULL for every handle).  Handles
 * not tuned yet are first tuned by pdf_autotune (5 launches per candidate).  rep:
 * steps taken, instances that reached their target (all handles), wall time.
 * Each handle must appear once.  Synchronous. */
int pdf_reconstruct_multi(int32_t n, pdf_handle* const* hs, int32_t n_iter, int32_t n_check,
                          int32_t start_given, void* const* alpha_dev,
                          const void* const* eps_true_dev, const double* const* target_err_dev,
                          int32_t* const* reached_iter_dev, double* const* best_err_dev,
                          int32_t* const* best_iter_dev, void* const* chi_cco_dev,
                          pdf_report* rep);

/* One Adam step (pdf_step) for each of n handles of any shapes, with the
 * caller's arrays of each (the entries have pdf_step's meaning for hs[i];
 * loss_dev may be NULL, or have NULL entries).  FP32 handles of one shape
 * class (grid, receiver and incidence tile counts) are advanced by one
 * grouped launch per kernel, the others one by one; the results equal n
 * separate pdf_step calls bit for bit.  Each handle must appear once.
 * Synchronous (the grouped launches' argument tables are built and released
 * in the call).  The message of a failure is in pdf_last_error(NULL). */
int pdf_step_multi(int32_t n, pdf_handle* const* hs, void* const* alpha_dev, void* const* m_dev,
                   void* const* v_dev, int32_t* const* t_dev, double* const* loss_dev);

/* FP64 method-of-moments synthesis of measured fields (Sec. 2.1, Eqs. 3-4):
 * solves (I - G_D X) E = E_inc on the support of chi = eps - 1 of a fine grid
 * and returns E_sca = G_S X E.  Stand-alone (no handle); synchronous.
 *   grid: the fine grid; eps_host: host complex128 [M][M] relative permittivity.
 *   esca_host: host complex128 [Ni][Ns] output.
 *   tol: relative residual of the iterative solve (e.g. 1e-10).
 * Errors: PDF_EINVAL, PDF_ENOMEM, PDF_EHIP, PDF_ENONFINITE (no convergence). */
int pdf_synthesize(const pdf_grid* grid, double freq_hz, const pdf_array* tx,
                   const pdf_array* rx, const double* eps_host, double tol,
                   double* esca_host, void* stream);

/* pdf_synthesize for n instances on one fine grid and frequency, each with its
 * own antenna positions (e.g. jittered), solved concurrently by `workers`
 * host threads (0: 8; at most 16) on streams of their own.  Synchronous.
 *   tx, rx: host arrays of n pdf_array each; every instance has the same
 *     Ni = tx[0].n and Ns = rx[0].n.
 *   eps_host: host complex128 [n][M][M]; esca_host: host complex128 [n][Ni][Ns].
 *   coarse: 0, or a divisor d of M: then jc_host (host complex128
 *     [n][Ni][M/d][M/d]) receives the induced currents chi E of the solution
 *     averaged over d x d pixel blocks (the currents on a d-times coarser grid).
 *   stream: used only for the shared tables (synchronised).
 * Errors as pdf_synthesize; the message names the first failing instance. */
int pdf_synthesize_batch(const pdf_grid* grid, double freq_hz, int32_t n, const pdf_array* tx,
                         const pdf_array* rx, const double* eps_host, double tol,
                         double* esca_host, int32_t coarse, double* jc_host, int32_t workers,
                         void* stream);

/* ------------------------------------------------------------------------
 * Warm-start network: an addition to the method (the paper has none).  A
 * fully connected network with exact GELU between its affine layers predicts
 * the start coefficients alpha_0 from the measured fields; it is trained on
 * pairs made by the FP64 MoM (pdf_synthesize_batch with coarse currents, then
 * pdf_analyze).  GEMM operands are bfloat16 (round to nearest even), with FP32
 * accumulation, biases, pre-activations, gradients, master weights and Adam
 * state (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *   Layer l (0 <= l < n_layers): z = h W_l^T + b_l with W_l FP32 [sizes[l+1]][sizes[l]]
 *   row-major, h_0 = s_in * x, h_{l+1} = gelu(z) for hidden layers, output
 *   y = s_out * z of the last layer.  All device arrays are row-major FP32.
 * The handle owns its buffers (sized for batch_max rows) and uses `stream`;
 * calls are asynchronous on it unless stated.  Errors: PDF_EINVAL, PDF_ENOMEM,
 * PDF_EHIP; the message is in pdf_last_error(NULL). */
typedef struct pdf_mlp pdf_mlp;

/* sizes: n_layers + 1 widths (input, hidden..., output).  Weights start at 0:
 * set every layer with pdf_mlp_set_layer.  Synchronous. */
int pdf_mlp_create(int32_t n_layers, const int32_t* sizes, int32_t batch_max, void* stream,
                   pdf_mlp** out);
/* Host FP32 weights and bias of layer l in; resets that layer's Adam state and
 * the step count.  Synchronous. */
int pdf_mlp_set_layer(pdf_mlp* net, int32_t l, const float* W_host, const float* b_host);
/* Layer l out to host FP32: what = 0 weights and bias, 1 their gradients from
 * the last pdf_mlp_train_step.  Synchronous. */
int pdf_mlp_get_layer(pdf_mlp* net, int32_t l, int32_t what, float* W_host, float* b_host);
/* y_dev [B][n_out] = s_out * net(s_in * x_dev [B][n_in]), 1 <= B <= batch_max. */
int pdf_mlp_forward(pdf_mlp* net, const float* x_dev, float s_in, float s_out, int32_t B,
                    float* y_dev);
/* One Adam step on the mean squared error over the B rows idx_dev[0..B) (device
 * int32, or NULL for rows 0..B) of x_dev [n_rows][n_in] against t_dev
 * [n_rows][n_out] (targets in the network's output units, i.e. before s_out).
 * Indices outside [0, n_rows) are clamped into it (callers should not pass
 * them).  loss_dev: device double, the batch MSE before the step (may be NULL). */
int pdf_mlp_train_step(pdf_mlp* net, const float* x_dev, const float* t_dev, int32_t n_rows,
                       const int32_t* idx_dev, float s_in, int32_t B, double lr,
                       double* loss_dev);
int pdf_mlp_widths(const pdf_mlp* net, int32_t* n_in, int32_t* n_out, int32_t* batch_max);
void pdf_mlp_destroy(pdf_mlp* net);

/* Start values of every instance of h (FP32 handles): the back-propagation
 * start of pdf_init_alpha (Sec. 3.1) and the network's prediction
 * s_out * net(s_in * E_sca) are both evaluated with the physics loss, and each
 * instance keeps the one with the lower total loss (so the network can only
 * replace a worse start).  The network maps the handle's E_sca [Ni][Ns]
 * (interleaved Re, Im: n_in = 2 Ni Ns) to alpha [Ni][K][K] (n_out = 2 Ni K^2).
 *   alpha_dev: [B][Ni][K][K] out.  chosen_dev: device int32 [B] out, 1 where
 *   the network's start was kept (may be NULL).  loss_dev: device double
 *   [B][2] out, total loss of the two starts (back-propagation, network), may
 *   be NULL.  Requires pdf_set_data. */
int pdf_warm_start(pdf_handle* h, pdf_mlp* net, float s_in, float s_out, void* alpha_dev,
                   int32_t* chosen_dev, double* loss_dev);

/* Kept Fourier coefficients of pixel currents (Sec. 2.3, Eq. 9): for n sets
 * of Ni currents J [n][Ni][M][M] on the handle's grid, alpha = F_T(J)
 * [n][Ni][K][K] with F_T the forward DFT divided by M^2 (so that the synthesis
 * F_T^* of alpha is the band-limited J).  Any n >= 1, independent of the
 * handle's batch. */
int pdf_analyze(pdf_handle* h, int32_t n, const void* J_dev, void* alpha_dev);

/* Coefficient network (Sec. 3.1, Fig. 4): instead of optimising alpha, a
 * fully connected network whose input is Re and Im of the start coefficients
 * alpha_0 predicts a correction,
 * alpha_hat = alpha_0 + s_out f_theta(s_in alpha_0), and
 * Adam (Sec. 3.3, the handle's lr, b1, b2, eps) trains its weights theta on
 * the loss at alpha_hat.  The paper's layer sizes are not available; here
 * every instance has its own network, shared by its Ni incidences: each
 * incidence is one row [Re alpha_0[i][:], Im alpha_0[i][:]] of width
 * D = 2 K^2 (modes in the [K][K] order), three dense layers D -> H -> H -> D,
 * tanh after the first two, output row [Re, Im] of Delta alpha[i][:] / s_out.
 * s_in = 1 / rms(alpha_0) and s_out = 1 / H give unit-scale inputs and a
 * first Adam step that moves alpha_hat about as far as a direct Adam step
 * moves alpha; s_in = s_out = 1 is the plain network (any finite values).
 * theta layout (handle precision, per instance, n_params values): per layer
 * a block of (in + 1) x out values, row-major [k][n], rows 0..in-1 the
 * weights (z[n] = sum_k x[k] W[k][n] + W[in][n]), row `in` the bias; the
 * blocks in layer order; instance b at theta + b * n_params.
 * Requires Ni <= 64 (PDF_EUNSUPPORTED otherwise) and 1 <= hidden <= 4096.
 * The library keeps a workspace of 4 B Ni H reals and B Ni K^2 complex
 * values in the handle (allocated on the first call, grown when needed). */
/* n_params out: values per instance.  Errors (PDF_EINVAL) leave their message
 * in pdf_last_error(NULL). */
int pdf_fcnn_size(const pdf_handle* h, int32_t hidden, int64_t* n_params);

/* alpha_hat_dev [B][Ni][K][K] out = alpha_0 + s_out f_theta(s_in alpha_0); alpha0_dev
 * the same shape, theta_dev [B][n_params].  alpha_hat must not alias alpha_0. */
int pdf_fcnn_forward(pdf_handle* h, int32_t hidden, double s_in, double s_out, const void* alpha0_dev,
                     const void* theta_dev, void* alpha_hat_dev);

/* One Adam step on theta in place: alpha_hat at the current weights (written
 * to alpha_hat_dev), loss and gradient there as in pdf_loss_grad (loss_dev as
 * there, may be NULL), the chain rule through the network, and the
 * bias-corrected update of every weight and bias.  m_dev, v_dev: moment
 * buffers of theta's shape, zero before step 1; t: this step's number,
 * counting from 1 (the bias corrections are fixed at launch, so a captured
 * graph of this call replays step t).  Requires pdf_set_data. */
int pdf_fcnn_step(pdf_handle* h, int32_t hidden, double s_in, double s_out, const void* alpha0_dev,
                  void* theta_dev, void* m_dev, void* v_dev, int32_t t, void* alpha_hat_dev, double* loss_dev);

/* Mean square (1/n) sum x_i^2 of n device reals (float for PDF_FP32, double
 * for PDF_FP64), FP64 accumulation in a fixed order, written to the device
 * double out_dev; asynchronous on `stream` (NULL: the default stream).  Used for the unit-RMS scales of
 * network inputs and outputs (the coefficient network of Sec. 3.1: s_in =
 * 1 / rms(alpha_0); the warm-start network's training data).  A complex array
 * is passed as 2n reals.  Errors (PDF_EINVAL: null, n < 1, bad precision)
 * leave their message in pdf_last_error(NULL). */
int pdf_mean_square(int32_t precision, int64_t n, const void* x_dev, double* out_dev, void* stream);

/* The linear pieces the loss is built from, applied alone to the handle's
 * whole batch (B instances x Ni incidences), for adjoint (dot-product) tests
 * of the device's own operators: the basis synthesis B = F_T^* (Sec. 2.3,
 * Eq. 9), the domain operator G_D as the 2x-padded FFT convolution (Sec. 2.1,
 * Eq. 3) and the receiver operator G_S (Sec. 2.1, Eq. 4), each through the
 * kernels of the loss-gradient pass (the adjoint ones through the adjoint
 * convolution with its analysis, and the G_S^H GEMM).
 *   op                    x_dev                     y_dev
 *   PDF_OP_SYNTH          alpha [B][Ni][K][K]       B alpha [B][Ni][M][M]
 *   PDF_OP_SYNTH_ADJ      [B][Ni][M][M]             B^H x [B][Ni][K][K]
 *   PDF_OP_GD             [B][Ni][M][M]             G_D x [B][Ni][M][M]
 *   PDF_OP_GD_SYNTH       alpha [B][Ni][K][K]       G_D B alpha [B][Ni][M][M]
 *   PDF_OP_GD_SYNTH_ADJ   [B][Ni][M][M]             B^H G_D^H x [B][Ni][K][K]
 *   PDF_OP_GS             [B][Ni][M][M]             G_S x [B][Ni][Ns]
 *   PDF_OP_GS_ADJ         [B][Ni][Ns]               G_S^H x [B][Ni][M][M]
 * B^H is the unnormalised forward DFT on the kept modes (M^2 F_T).  x and y
 * are device arrays in the handle's precision and must not alias.  Overwrites
 * the handle's per-iteration scratch (not alpha, Adam state or the data).
 * Errors: PDF_EINVAL (null, aliasing, unknown op). */
enum {
  PDF_OP_SYNTH = 0,
  PDF_OP_SYNTH_ADJ = 1,
  PDF_OP_GD = 2,
  PDF_OP_GD_SYNTH = 3,
  PDF_OP_GD_SYNTH_ADJ = 4,
  PDF_OP_GS = 5,
  PDF_OP_GS_ADJ = 6
};
int pdf_apply(pdf_handle* h, int32_t op, const void* x_dev, void* y_dev);

/* Per-kernel timing with HIP events recorded on the handle's stream around
 * each kernel of pdf_loss_grad / pdf_step (for benchmarks).  enable != 0
 * clears the record and starts recording up to max_steps iterations; 0 stops.
 * pdf_timing_read synchronises the stream and writes, for each of the
 * PDF_NKERNELS kernels of one iteration, the average duration in ms
 * (avg_ms[k]) over the recorded iterations; *n_steps gets their count.
 * Kernel order: 0 fwd_conv, 1 pixel_reduce, 2 image_reg, 3 adj_gemm, 4 adj_conv. */
#define PDF_NKERNELS 5
int pdf_timing(pdf_handle* h, int32_t enable, int32_t max_steps);
int pdf_timing_read(pdf_handle* h, double* avg_ms, int32_t* n_steps);

/* Release everything the handle owns (waits for its stream).  NULL is a no-op. */
void pdf_destroy(pdf_handle* h);

/* Message of the last failed call on h (or of the last failed pdf_setup /
 * pdf_tables_host / pdf_synthesize when h is NULL).  Never NULL. */
const char* pdf_last_error(const pdf_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* PDF_H */
