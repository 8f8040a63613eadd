/*
 * sht.h - C ABI of the Clenshaw-Curtis spherical-harmonic transform library
 * for AMD Instinct MI355X (gfx950).
 *
 * The transform pair is the one of Hotta & Ujiie, "A nestable,
 * multigrid-friendly grid on a sphere for global spectral models based on
 * Clenshaw-Curtis quadrature":
 *   synthesis (Sec. 2, eq. iSHT / eq. iLT): a Legendre sum per zonal
 *     wavenumber m, X^m(phi_j) = sum_n a_n^m P~_n^m(sin phi_j), followed by the
 *     zonal inverse DFT  x(lambda_i, phi_j) = sum_{m=-N..N} X^m e^{i m lambda_i};
 *   analysis (Sec. 2, eq. dSHT / eq. dLT / eq. dFT, discretised with the
 *     Clenshaw-Curtis rule of Sec. 3.1, eq. cc-quad / eq. cc-wgt): the zonal
 *     DFT X^m(phi_j) = (1/I) sum_i x e^{-i m lambda_i}, then the quadrature
 *     a_n^m = sum_j w_j P~_n^m(sin phi_j) X^m(phi_j), exact when J >= 2N+1
 *     (eq. cc-condition) and I > 2N (eq. fourier-condition).
 * The Legendre sums use the equatorial parity fold of App. B (eqs. B3, B4).
 *
 * Conventions
 *   Grids (sht_grid_t): SHT_GRID_FEJER2 is the paper's pole-free grid,
 *   theta_j = j*pi/(J+1), j = 1..J (Sec. 3.1, eq. cc-points);
 *   SHT_GRID_CC_POLES is the classical Clenshaw-Curtis grid with the poles,
 *   theta_j = j*pi/(J-1), j = 0..J-1; SHT_GRID_FEJER1 is the shifted grid
 *   of Sec. 3.3, theta_j = (j-1/2)*pi/J, j = 1..J (eq. fejer1-points), with
 *   Fejer's first-rule weights (eq. fejer1-wgt read with a factor 2 before
 *   its sum, without which the rule is not interpolatory); it does not
 *   nest.  Row 0 is nearest the north pole.
 *   lambda_i = 2*pi*i/I.  P~_n^m has unit L2 norm over mu in [-1, 1]
 *   (eq. pnm-ortho) and no Condon-Shortley phase.
 *
 * Memory layout (all buffers are device memory, contiguous, row-major):
 *   grid: [nfields][J][I] real;
 *   spec: [nfields][ncoef][2] (re, im), ncoef = (N+1)(N+2)/2, m-major:
 *         index(m, n) = m*(2N+3-m)/2 + (n-m), 0 <= m <= n <= N.
 *         Im of m = 0 is written as 0 and ignored on input.
 *   Element type: double for SHT_FORM_FP64, float for SHT_FORM_FP32 and
 *   SHT_FORM_BF16X6 (that form splits operands into bfloat16 pieces inside
 *   the Legendre kernels; its inputs and outputs are float).
 *   Multi-level plans: the buffers of the levels are concatenated in level
 *   order (use SHT_Q_GRID_OFFSET / SHT_Q_SPEC_OFFSET to find a level).
 *
 * Ownership and concurrency
 *   The caller owns every grid and spec buffer.  The plan owns its tables,
 *   twiddles and workspace.  sht_forward / sht_inverse / the adjoints
 *   allocate nothing, do not synchronise with the host and only enqueue work
 *   on `stream` (a hipStream_t; NULL is the default stream).  A plan holds
 *   one workspace, so two calls on the same plan must not overlap in time
 *   (use one stream per plan, or one plan per stream).  Inputs and outputs
 *   must not alias.  Input buffers are not modified.
 *
 * Errors
 *   Every entry point returns SHT_OK (0) or a negative code; the message of
 *   the last failure on the calling thread is available from
 *   sht_last_error().  Arguments are validated before any work is enqueued.
 *   No C++ exception crosses this interface.
 */
#ifndef SHT_H_
#define SHT_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sht_plan_s* sht_plan_t;

typedef enum {
  SHT_GRID_CC_POLES = 0,
  SHT_GRID_FEJER2 = 1,
  SHT_GRID_FEJER1 = 2,
  SHT_GRID_GAUSS = 3   /* Gaussian grid (Sec. 2): the paper's comparison
                          grid, for reference transforms (exact when
                          J >= N+1) */
} sht_grid_t;

typedef enum {
  SHT_FORM_FP64 = 0,   /* FP64 data, FP64 MFMA (v_mfma_f64_16x16x4) */
  SHT_FORM_FP32 = 1,   /* FP32 data, FP32 MFMA (v_mfma_f32_16x16x4) */
  SHT_FORM_BF16X6 = 2  /* FP32 data; Legendre operands split into three
                          bfloat16 pieces, six piece products per term,
                          FP32 accumulation */
} sht_form_t;

typedef struct {
  int grid;       /* sht_grid_t */
  int form;       /* sht_form_t */
  int autotune;   /* nonzero: time candidate tile shapes at plan time */
  int use_graph;  /* nonzero: replay each transform from a captured hipGraph */
  int reduced;    /* nonzero: reduced transform (Sec. 4.1): for each m the
                     polar latitudes at which every |P~_n^m| (n = m..N) is
                     below 1e-16 are left out of both Legendre sums, in
                     whole blocks of the kernels (32 latitudes; 16 in the
                     FP64 analysis; 128 in the synthesis).  The terms left
                     out are below 1e-16 relative. */
  int otf;        /* nonzero (any form; not with reduced or autotune):
                     both Legendre kernels generate P~_n^m by the three-term
                     recurrence (Sec. 4.1), in FP64, from two stored FP64
                     seed rows per 16 degrees instead of reading a table,
                     and round it once to the form's element type; the plan
                     keeps no table (seed rows: 1/8 of the table's entries,
                     in FP64). */
  int zonal;      /* sht_zonal_t: how a multi-level plan launches its zonal
                     stage (Sec. 3.2: a hierarchy of truncations batched in
                     one plan).  Single-level plans ignore it. */
} sht_options;

typedef enum {
  SHT_ZONAL_AUTO = 0,        /* per direction: with autotune, whichever of
                                the two below timed faster at plan time;
                                without, one launch where the levels allow
                                it and the one-launch kernel of the form and
                                direction runs without register spills */
  SHT_ZONAL_ONE_LAUNCH = 1,  /* one persistent launch over every level's
                                work items where every level has I = 400,
                                800 or 1600 or I <= 1024 (else as below) */
  SHT_ZONAL_PER_LENGTH = 2   /* one launch per compile-time FFT length and
                                one for the other levels */
} sht_zonal_t;

enum {
  SHT_OK = 0,
  SHT_EINVAL = -1,   /* bad argument */
  SHT_ENOMEM = -2,   /* device or host allocation failed */
  SHT_EHIP = -3,     /* a HIP runtime call failed */
  SHT_ESTATE = -4    /* destroyed or corrupt plan handle */
};

/* Query keys for sht_plan_query. */
enum {
  SHT_Q_NLEVELS = 0,        /* int */
  SHT_Q_NCOEF = 1,          /* int, level 0 */
  SHT_Q_EXACT = 2,          /* int: 1 if J >= 2N+1 on every level */
  SHT_Q_WORKSPACE_BYTES = 3,/* size_t */
  SHT_Q_TABLE_BYTES = 4,    /* size_t */
  SHT_Q_GRID_ELEMS = 5,     /* size_t: elements of the (concatenated) grid */
  SHT_Q_SPEC_ELEMS = 6,     /* size_t: elements of the (concatenated) spec */
  SHT_Q_FORM = 7,           /* int */
  SHT_Q_GRID_KIND = 8,      /* int */
  SHT_Q_LEGENDRE_FLOPS = 9, /* double: parity-folded Legendre flops of one
                               direction, 2*ceil(J/2)*(N+1)(N+2)*F summed
                               over levels */
  SHT_Q_LEGENDRE_FLOPS_KEPT = 10, /* double: the part of SHT_Q_LEGENDRE_FLOPS
                               the analysis kernel multiplies when the plan
                               uses the reduced transform: for each m,
                               4 (N-m+1) F (ceil(J/2) - b_m), b_m = the latitudes
                               left out, a whole number of the kernel's
                               blocks (32; 16 in the FP64 form); equal to
                               SHT_Q_LEGENDRE_FLOPS otherwise */
  SHT_Q_ZONAL_ONE_LAUNCH = 11, /* int, multi-level plans: bit 0 set if the
                               zonal analysis runs as one launch over all
                               levels, bit 1 the zonal synthesis (see
                               sht_zonal_t); 0 for single-level plans */
  SHT_Q_GRID_OFFSET = 100,  /* size_t: element offset of level (key-100) */
  SHT_Q_SPEC_OFFSET = 200   /* size_t: element offset of level (key-200) */
};

/*
 * sht_plan: plan for one level with the defaults (SHT_GRID_CC_POLES,
 * SHT_FORM_FP64) on the current HIP device.  Returns NULL on failure.
 *   N >= 0 truncation wavenumber; J latitudes (>= 2 on CC_POLES, >= 1 on
 *   FEJER2, FEJER1 and GAUSS); I >= 2N+1 longitudes (radix 2, 3, 5 only, I <= 4096);
 *   nfields >= 1 independent fields.  J < 2N+1 is accepted (the quadrature
 *   then aliases, Sec. 3.1; SHT_Q_EXACT reports 0).
 * Plan time builds the nodes and weights (Sec. 3.1, eq. cc-points,
 * eq. cc-wgt; App. A), the table of P~_n^m (three-term recurrence of
 * Sec. 4.1, evaluated with a separately carried binary exponent so that no
 * value underflows) and uploads them; it synchronises the device.
 */
sht_plan_t sht_plan(int N, int J, int I, int nfields);

/* As sht_plan with options (NULL = defaults); the plan goes to *out. */
int sht_plan_ex(int N, int J, int I, int nfields, const sht_options* opts,
                sht_plan_t* out);

/*
 * A hierarchy of nlevels (1..8) independent transforms executed together
 * (e.g. the nested truncations of Sec. 3.2): one Legendre launch per
 * direction covers all levels; the zonal stage launches once per level
 * whose I has a compile-time FFT plan and once for all other levels.
 * Arrays have nlevels entries; buffers are concatenated.
 */
int sht_plan_multi(int nlevels, const int* N, const int* J, const int* I,
                   const int* nfields, const sht_options* opts,
                   sht_plan_t* out);

/* Analysis, grid -> spec (Sec. 2 eq. dSHT; Sec. 3.1 eq. cc-quad). */
int sht_forward(sht_plan_t plan, const void* grid, void* spec, void* stream);

/*
 * sht_forward_noalloc: the analysis of sht_forward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  It runs the same kernels with the
 * plan's zonal-to-Legendre workspace replaced by a static device array of
 * SHT_NOALLOC_WORKSPACE_BYTES (64 MiB) that the library holds on every GPU
 * it runs on until the process ends; it calls no hipMalloc, hipFree, event,
 * graph or allocating library routine (a plan built with use_graph runs
 * eagerly here).  The caller passes the plan (built beforehand), the grid
 * and the spec as for sht_forward; the result equals sht_forward's.
 * Every call on one GPU shares that GPU's array, and each call first clears
 * the part that must start at zero: calls that overlap in time on one GPU
 * (on different streams, or from different threads) race and must be
 * ordered by the caller.  Errors: as sht_forward; SHT_EINVAL if the plan's
 * workspace (SHT_Q_WORKSPACE_BYTES) exceeds SHT_NOALLOC_WORKSPACE_BYTES or
 * the plan belongs to another device than the current one.
 */
#define SHT_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
int sht_forward_noalloc(sht_plan_t plan, const void* grid, void* spec, void* stream);

/* Synthesis, spec -> grid (Sec. 2 eq. iSHT, eq. iLT). */
int sht_inverse(sht_plan_t plan, const void* spec, void* grid, void* stream);

/*
 * Transpose of sht_forward under the Euclidean inner product of the stored
 * real arrays: grid_bar = forward^T spec_bar.  Equals (w_j / I) times a
 * synthesis of spec_bar with every m > 0 coefficient halved and Im of m = 0
 * dropped.  (Not a formula of the paper; it is what reverse-mode
 * differentiation of the analysis needs.)
 */
int sht_forward_adjoint(sht_plan_t plan, const void* spec_bar, void* grid_bar,
                        void* stream);

/*
 * Transpose of sht_inverse: spec_bar = inverse^T grid_bar, i.e. c_m * I times
 * an analysis without the weights w_j, c_0 = 1, c_m = 2 (m > 0), and Im of
 * m = 0 set to 0.
 */
int sht_inverse_adjoint(sht_plan_t plan, const void* grid_bar, void* spec_bar,
                        void* stream);

/* Read a plan property (see SHT_Q_*); `out` points to the documented type. */
int sht_plan_query(sht_plan_t plan, int key, void* out);

/*
 * Copy plan tables of level 0 to host memory (any pointer may be NULL):
 * mu[J] = sin(latitude) of each row, w[J] quadrature weights, and
 * alf[(N+1)(N+2)/2 * ceil(J/2)] = P~_n^m(mu_j) for the northern rows
 * j < ceil(J/2), in spec order (m-major), each entry a row of ceil(J/2)
 * values, as built in FP64 before any conversion to the form's precision.
 */
int sht_plan_tables(sht_plan_t plan, double* mu, double* w, double* alf);

/*
 * Per-stage timing for measurement.  While enabled, every transform call
 * brackets each of its kernel launches with hipEvents recorded on the
 * caller's stream (stages: 0 zonal analysis, 1 Legendre analysis,
 * 2 Legendre synthesis, 3 zonal synthesis).  sht_plan_profile_read waits for
 * the last recorded event, returns the summed milliseconds ms[4] and launch
 * counts counts[4] since the last read (or enable), and starts over.
 * Profiling creates events on first use, so keep it off under graph capture.
 */
int sht_plan_profile(sht_plan_t plan, int enable);
int sht_plan_profile_read(sht_plan_t plan, double* ms, int* counts);

/* Release every resource of the plan (after the device has finished with
 * any work that uses it).  A destroyed handle is rejected with SHT_ESTATE. */
int sht_plan_destroy(sht_plan_t plan);

/* Message for the last failure on the calling thread ("" if none). */
const char* sht_last_error(void);

/*
 * Device bytes held by all live plans of the process (tables, workspaces,
 * schedules), written to *out.  A plan whose construction fails frees what
 * it had allocated, so this is unchanged by a failed sht_plan_ex.  The
 * environment variable SHT_TEST_MAX_BYTES, when set, caps this total: a plan
 * whose allocations would exceed it fails with SHT_ENOMEM (for tests of the
 * out-of-memory path).  SHT_EINVAL if out is NULL.
 */
int sht_device_bytes(size_t* out);

/*
 * Transfers for multigrid cycles (App. C: restriction and prolongation
 * between a finer and a coarser level), enqueued on `stream`; no plan
 * needed.  dbl nonzero: double elements, else float.  Buffers are device
 * memory, 16-byte aligned, caller-owned, and must not overlap.
 *
 * sht_spec_retruncate: spectral restriction (N_out < N_in) or prolongation
 *   (N_out > N_in) of nfields spectra in the layout of sht_forward:
 *   out(m, n) = in(m, n) for n <= min(N_in, N_out), 0 for n > N_in.
 * sht_grid_inject: grid restriction by injection (Sec. 3.2, App. C): the
 *   coarse grid's rows and columns are a subset of the fine grid's.
 *   SHT_GRID_CC_POLES: (J_fine-1) = s (J_coarse-1), coarse row j = fine row
 *   s j; SHT_GRID_FEJER2: (J_fine+1) = s (J_coarse+1), coarse row j = fine
 *   row s (j+1) - 1; columns: I_fine = t I_coarse, coarse column i = fine
 *   column t i.  SHT_GRID_FEJER1 does not nest (SHT_EINVAL).  fine and
 *   coarse need only be element-aligned (one level's slice of a multi-level
 *   plan's concatenated grids).
 * Both return SHT_EINVAL on bad sizes or pointers, SHT_EHIP on a launch
 * failure.
 */
int sht_spec_retruncate(int N_in, int N_out, int nfields, int dbl,
                        const void* spec_in, void* spec_out, void* stream);
int sht_grid_inject(int J_fine, int I_fine, int J_coarse, int I_coarse,
                    int nfields, int grid, int dbl, const void* fine,
                    void* coarse, void* stream);

/*
 * Pointwise product of n grid values, out[i] = a[i] * b[i] (the quadratic
 * and cubic terms whose aliasing Sec. 4.2 measures); out may be a or b.
 * Same conventions as the transfers above.
 */
int sht_grid_product(long long n, int dbl, const void* a, const void* b,
                     void* out, void* stream);

/*
 * The two pieces of the residual R = (I - dt/2 L) X - F of the elliptic
 * problem of App. C (eq. elliptic), for a variable-coefficient Laplacian
 * L X = kappa * lap(X) evaluated pseudo-spectrally: analyse X, apply the
 * spectral Laplacian, synthesise, then the grid update.  Same conventions
 * as the transfers above.
 *
 * sht_spec_laplacian: out(m, n) = c_n in(m, n) with c_n = -scale n (n+1)
 *   (computed in double, rounded once to the element type): the Laplacian
 *   on a sphere of radius 1/sqrt(scale), for nfields spectra of truncation
 *   N in the layout of sht_forward.  out may equal in.
 * sht_grid_residual: r[i] = x[i] - alpha * kappa[i mod n_per] * y[i] - f[i]
 *   for i < n (n a multiple of n_per: kappa is one grid of n_per values
 *   shared by all fields).  r may equal x, y or f.
 * Unlike the calls above, these two take element-aligned buffers (one
 * level's slice of a multi-level plan's concatenated grids or spectra):
 * sht_spec_laplacian needs in and out aligned to a complex pair (8 bytes
 * for float, 16 for double), sht_grid_residual to one element.
 * SHT_EINVAL on bad sizes, a non-finite scale or alpha, or bad pointers;
 * SHT_EHIP on a launch failure.
 */
int sht_spec_laplacian(int N, int nfields, int dbl, double scale,
                       const void* in, void* out, void* stream);
int sht_grid_residual(long long n, long long n_per, int dbl, double alpha,
                      const void* x, const void* kappa, const void* y,
                      const void* f, void* r, void* stream);

/*
 * Host-only planning (no GPU needed): nodes and weights of a grid, and the
 * FP64 table of P~_n^m for the northern rows, as sht_plan_tables.  Returns
 * SHT_EINVAL on bad arguments.
 */
int sht_host_tables(int N, int J, int grid, double* mu, double* w,
                    double* alf);

#ifdef __cplusplus
}
#endif

#endif /* SHT_H_ */
