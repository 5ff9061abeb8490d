/*
 * hh.h -- C ABI of the MI355X (gfx950) hierarchical-homogenization library.
 *
 * Computes effective elastic stiffnesses of segmented 3-D images by the
 * periodic FFT (Fourier-Galerkin) elasticity solve of the paper's Appendix A,
 * averaged over a region as in Sec. 4, and the two-level hierarchical scheme
 * of Sec. 3 with the n^-1 extrapolation of Sec. 5 (eq_fit_power_law).
 *
 * Conventions (all entry points):
 *  - Images are C-contiguous arrays indexed [z][y][x] (x fastest); tensor
 *    index 1/2/3 is x/y/z.  Sizes are in voxels; moduli in GPa.
 *  - Stiffness matrices are 6x6 Voigt matrices, row-major, in the order
 *    (11, 22, 33, 23, 13, 12), acting on strain vectors with engineering
 *    shear components (2 eps_ij); an isotropic phase has C44 = G.
 *  - "21 components" is the upper triangle of a symmetric 6x6, row-major.
 *  - Pointers flagged *_on_device are device pointers of the context's
 *    device; all others are host pointers.  The caller owns every buffer it
 *    passes; the library owns its workspace and returns no allocations.
 *  - Return value: HH_OK (0) or a negative HH_E* code; hh_last_error()
 *    describes the last failure on that context.  No exception crosses the
 *    ABI.  A context is not thread-safe: use one per host thread / stream.
 *  - Calls are synchronous with respect to the host: outputs are written
 *    when the call returns.  Device work runs on the context's stream.
 */
#ifndef HH_H
#define HH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HH_OK 0
#define HH_EINVAL (-1)        /* bad sizes / arguments, label >= nphase, N % n != 0, ... */
#define HH_EUNSUPPORTED (-2)  /* axis length without compiled FFT passes (see hh_size_supported) */
#define HH_ENOMEM (-3)        /* device allocation failed */
#define HH_EDEVICE (-4)       /* HIP runtime error or not a gfx950 device */
#define HH_ESINGULAR (-5)     /* averaged strain matrix E_R not invertible */
#define HH_ENOCONV (-6)       /* max_iter reached: best C still written, report.status set */
#define HH_ESTAGNATED (-7)    /* residual stopped decreasing (e.g. tol below FP32 floor) */
#define HH_EBREAKDOWN (-8)    /* (p, A p) <= 0 or non-finite values in the iteration */

#define HH_NKERNEL 8          /* kernel classes timed in hh_report.kernel_ms */
#define HH_NVARIANT 5         /* compiled tile variants per FP32 axis length */
/* kernel class indices */
#define HH_K_ZINV 0
#define HH_K_YINV 1
#define HH_K_X 2
#define HH_K_YFWD 3
#define HH_K_ZFWD 4
#define HH_K_FIN 5
#define HH_K_SETUP 6
#define HH_K_OTHER 7

typedef struct hh_ctx hh_ctx;

/* Isotropic phase: bulk modulus K and shear modulus G (both > 0), Sec. 4. */
typedef struct {
  double K, G;
} hh_phase;

/* Solver options.  hh_default_opts() fills the defaults given here. */
typedef struct {
  double tol;        /* stop when ||r|| <= tol ||b||, r = -G*(C:(E+eps*)); default 1e-6 */
  int max_iter;      /* per load case; 0 (default) = from the phase contrast kappa (largest
                        over smallest eigenvalue 3K or 2G of the phase stiffnesses):
                        max(1000, ceil(sqrt(kappa) ln(2 / tol))), twice the classical
                        conjugate-gradient bound; 1000 for anisotropic voxels */
  int scheme;        /* 0: conjugate gradients (Appendix A); 1: basic fixed point with
                        reference medium (ref_lambda, ref_mu); default 0 */
  int precision;     /* 0: FP32 fields and FFTs, FP64 reductions/scalars/averages;
                        1: FP64 throughout; default 0 */
  int nyquist;       /* even axes: 0 = Nyquist wavenumber component set to 0;
                        1 = operator zero at every frequency with a Nyquist component */
  int profile;       /* 1: time every kernel class with HIP events (hh_report.kernel_ms) */
  int stall_limit;   /* iterations without a new smallest residual before
                        HH_ESTAGNATED; 0 (default) = max(100, ceil(sqrt(kappa))),
                        100 for anisotropic voxels */
  int chunk;         /* iterations launched between convergence polls; default 8 */
  double ref_lambda, ref_mu; /* basic scheme reference medium; <= 0: mid-range of the phases */
  int tune;          /* FP32: 1 = the first solve of a shape in a context times the compiled
                        tile variants of each pass (on that group's own buffers, before its
                        right-hand side) and the context keeps the fastest; 0 = default
                        tiles; default 1 */
  int graph;         /* 1 = each chunk of iterations is captured once as a hipGraph and
                        replayed (not with profile); 0 = plain launches; default 1 */
  int plan[3];       /* tile variant forced for the z, y and x passes (0..HH_NVARIANT-1,
                        FP64: 0 only); -1 = tuned or default; default -1 */
  int loads_per_wave; /* 1..6: the load cases of an image are solved at most this many at
                        a time (the others wait for device memory), and images then run
                        one at a time; 0 = all six together unless the six systems of one
                        image do not fit in device memory, then as many as fit; default 0 */
  int retry;         /* 1 (default): with FP32 fields, an image of isotropic phases whose
                        solve stops with HH_ESTAGNATED or HH_EBREAKDOWN (the FP32 floor, e.g.
                        at extreme phase contrast) is solved again with FP64 fields when its axis
                        lengths have FP64 passes, with at least the contrast-derived stall
                        limit; hh_report.retried counts them; 0 = off */
  int verify;        /* 1: hh_homogenize also solves the image with FP64 fields at tol
                        1e-10 and reports the difference in hh_report.err_vs_oracle;
                        default 0 */
  int lanes;         /* hh_homogenize_batch: shape groups solved concurrently, each on its
                        own stream, host thread and workspace (1..4; 0 = default = 1, one
                        group after another; profile forces 1); results do not depend on it */
} hh_opts;

/* Per-call report. */
typedef struct {
  int status;                   /* HH_OK or the worst per-load status */
  int iters[6];                 /* iterations per load (first item for batched calls) */
  double rel_resid[6];          /* final ||r|| / ||b|| per load (first item) */
  double asym;                  /* max |C - C^T| / max |C| of the raw Sigma E^-1 */
  double seconds;               /* device wall time of the call (HIP events) */
  double voxel_iters;           /* sum over items and loads of voxels x iterations */
  long long items;              /* images homogenized by the call */
  double kernel_ms[HH_NKERNEL]; /* with opts.profile: summed device time per class */
  int kernel_launches[HH_NKERNEL];
  int plan[3];                  /* tile variants (z, y, x) of the last group solved */
  double setup_ms;              /* host time spent tuning and building graphs in the call
                                   (one-time per shape / argument set; part of seconds) */
  long long retried;            /* images solved again with FP64 fields (hh_opts.retry) */
  double bytes_moved;           /* algorithmic device-memory bytes of the solver passes: per
                                   system iteration 63 complex words per half-spectrum
                                   frequency (zinv 15, y 12 + 12, x 12, zfwd 12) plus the
                                   labels (or 21 stiffness words per voxel), and 27 words per
                                   frequency for the right-hand side */
  double err_vs_oracle;         /* with hh_opts.verify (hh_homogenize): relative difference,
                                   ||C - C64||_F / ||C64||_F on Mandel-scaled matrices, from
                                   the same solve with FP64 fields at tol 1e-10 (that path
                                   matches the FP64 CPU oracle to 1e-8 in the tests); -1 when
                                   not computed */
} hh_report;

/* Fills *opts with the defaults listed in hh_opts. */
void hh_default_opts(hh_opts *opts);

/* Creates a context on HIP device `device`, launching on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Fails with HH_EDEVICE if the
 * device is not gfx950. */
int hh_create(hh_ctx **ctx, int device, void *hip_stream);
/* Changes the stream of an existing context. */
int hh_set_stream(hh_ctx *ctx, void *hip_stream);
/* Frees the context and its device workspace.  NULL is ignored. */
void hh_destroy(hh_ctx *ctx);
/* Message describing the last failing call on ctx (empty if none); with
 * ctx = NULL, the reason the last hh_create of the calling thread failed. */
const char *hh_last_error(const hh_ctx *ctx);
/* Device workspace currently held by the context, in bytes. */
long long hh_workspace_bytes(const hh_ctx *ctx);
/* Releases the context's workspace (it is re-allocated on demand). */
void hh_release_workspace(hh_ctx *ctx);
/* 1 if axis length n has compiled FFT passes at `precision`, else 0.  The
 * list is fixed at build time.
 * FP32 (precision 0): 2 3 4 5 6 8 9 10 12 15 16 18 20 24 25 27 30 32 36 40
 * 45 48 50 60 64 70 72 75 80 85 90 95 96 100 110 115 120 128 130 140 144
 * 150 160 170 180 190 192 200 220 225 235 240 245 256 265 272 288 300 310
 * 320 340 512 900 1024
 * (among them the boxes of the paper's subimage sizes of Sec. 5 with 5, 10
 * or 20 voxels of padding per side, and a plain 900^3 solve).
 * FP64 (precision 1): 2 3 4 5 6 8 9 10 12 15 16 18 20 24 25 27 30 32 36 40
 * 45 48 60 64 80 85 95 96 100 110 120 128 144 150 160 192 256. */
int hh_size_supported(int n, int precision);

/*
 * Effective stiffness of one label image (Sec. 4; Appendix A solve).
 * labels: uint8[nz][ny][nx] phase indices < nphase.  phases[nphase].
 * loads: 6x6, column a = the engineering-Voigt macroscopic strain of load a
 *   (column-major, loads[6*a + i]); NULL = the six unit strains.  The six
 *   loads must be independent.
 * region: {x0, y0, z0, x1, y1, z1}, half open, the averaging region
 *   Omega_R inside the periodic box; NULL = the whole box.
 * C_out: symmetrized (C + C^T)/2 of C_R = Sigma_R E_R^-1, 36 doubles.
 * C_raw: the raw C_R (may be NULL).  report: may be NULL.
 * The six load cases run together; when their six systems (about 52 GB
 * each at 1024^3 in FP32) do not fit in device memory they run a few at a
 * time (hh_opts.loads_per_wave), with the same result.
 */
int hh_homogenize(hh_ctx *ctx, const uint8_t *labels, int nx, int ny, int nz, int labels_on_device,
                  const hh_phase *phases, int nphase, const double *loads, const int *region,
                  const hh_opts *opts, double C_out[36], double C_raw[36], hh_report *report);

/*
 * hh_homogenize for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one label image already on the device, the six unit loads,
 * the whole box as region.  Its buffers come from a static device array of
 * 128 MiB that the library holds on every GPU it runs on until the process
 * ends (enough for FP32 images up to about 64^3; larger images return
 * HH_EINVAL before any device work).  It calls no hipMalloc or hipFree and
 * no allocating library routine, and launches plainly (opts.graph, profile,
 * retry, verify and lanes are ignored).  All calls on one GPU share that
 * array: calls that overlap on one GPU, from any context or thread, race.
 * The array keeps the last call's contents; every call clears what must
 * start at zero.  Arguments and results as in hh_homogenize.
 */
int hh_homogenize_noalloc(hh_ctx *ctx, const uint8_t *labels_device, int nx, int ny, int nz,
                          const hh_phase *phases, int nphase, const hh_opts *opts, double C_out[36],
                          hh_report *report);

/*
 * Effective stiffness of an image of anisotropic voxels (the intermediate
 * image of Sec. 3, solved as stated at the end of Sec. 4).
 * C21: per voxel 21 upper-triangle components, [nz][ny][nx][21] doubles
 *   (host or device); each voxel stiffness must be positive definite.
 */
int hh_homogenize_aniso(hh_ctx *ctx, const double *C21, int nx, int ny, int nz, int c21_on_device,
                        const hh_opts *opts, double C_out[36], double C_raw[36], hh_report *report);

/*
 * Batch of independent images of possibly different sizes and phase sets
 * (the subimage solves of Sec. 3 are independent).  Item i has shape
 * dims[3*i .. 3*i+2] = (nx, ny, nz), labels at byte
 * offset label_off[i] of `labels` (uint8, [z][y][x]), phases
 * phases[phase_off[i] .. phase_off[i] + nphase[i]), and averaging region
 * regions[6*i ..] (NULL = whole boxes).  Items of equal shape are solved in
 * one launch per pass.  C_out: nitems x 36 symmetrized stiffnesses;
 * C_raw: nitems x 36 raw (may be NULL); item_status: nitems HH codes (may be
 * NULL); item_iters: nitems x 6 iteration counts (may be NULL).
 */
int hh_homogenize_batch(hh_ctx *ctx, int nitems, const int *dims, const uint8_t *labels,
                        long long labels_bytes, int labels_on_device, const long long *label_off,
                        const hh_phase *phases, const int *phase_off, const int *nphase,
                        const int *regions, const hh_opts *opts, double *C_out, double *C_raw,
                        int *item_status, int *item_iters, hh_report *report);

/*
 * Two-level hierarchical homogenization (Sec. 3, Fig. 2; padding Sec. 4,
 * Fig. 4).  labels: uint8[nz][ny][nx]; n_sub must divide each dimension and
 * 2 pad < each dimension.  Each n_sub^3 block is solved in the box
 * extended by `pad` voxels of surrounding material (periodic wrap at the
 * image edge) and averaged over the block; the symmetrized block stiffnesses
 * form the intermediate image, which is solved with anisotropic voxels.
 * C_out: final C* (36).  C_sub: (nz/n)(ny/n)(nx/n) x 21 symmetrized block
 * stiffnesses, C order (may be NULL).  use_surrogate = 1 takes the subimage
 * stiffnesses from the networks attached with hh_set_surrogate, with their
 * gate and the FFT solve as fallback (hh_hierarchical_surrogate without the
 * fallback flags); HH_EINVAL when none are attached.  With one subimage (n = image size)
 * the intermediate image is a single voxel and C* is its stiffness; an
 * intermediate image with some axes of length 1 and others longer returns
 * HH_EUNSUPPORTED.
 */
int hh_hierarchical(hh_ctx *ctx, const uint8_t *labels, int nx, int ny, int nz, int labels_on_device,
                    const hh_phase *phases, int nphase, int n_sub, int pad, int use_surrogate,
                    const hh_opts *opts, double C_out[36], double *C_sub, hh_report *report);

/*
 * Repeated coarse-graining: the scheme of Sec. 3 applied again to its own
 * intermediate image (the renormalization the paper's scheme is modelled
 * on), nlevels times before the final solve.  Level 1 is hh_hierarchical's
 * first step on the label image with blocks n_sub[0] and padding pad[0].
 * Level l > 1 cuts the current intermediate image (21-component
 * symmetrized stiffnesses) into n_sub[l-1]^3 blocks, solves each in the box
 * extended by pad[l-1] voxels (periodic wrap) with anisotropic voxels,
 * averages over the block, and assembles the symmetrized results into the
 * next intermediate image.  The last image is solved whole (or, when it is a
 * single voxel, is C*).  nlevels = 1 gives hh_hierarchical's C*.  Every
 * n_sub[l] must divide its image, 2 pad[l] < that image's edges, and every
 * box edge and the last image's edges must be compiled lengths.
 * report.items counts level-1 subimages; report.voxel_iters sums all levels.
 */
int hh_hierarchical_levels(hh_ctx *ctx, const uint8_t *labels, int nx, int ny, int nz, int labels_on_device,
                           const hh_phase *phases, int nphase, const int *n_sub, const int *pad, int nlevels,
                           const hh_opts *opts, double C_out[36], hh_report *report);

/*
 * Partition + padding of the two-level scheme (Sec. 3; Sec. 4, Fig. 4) on
 * its own: copies every n_sub^3 block of the [nz][ny][nx] image, extended by
 * `pad` voxels of surrounding material (periodic wrap at the image edge),
 * into pack_device as (nz/n)(ny/n)(nx/n) consecutive boxes of
 * (n_sub + 2 pad)^3 bytes, blocks in C order.  pack_device: device buffer
 * owned by the caller of at least that size.
 */
int hh_gather_subimages(hh_ctx *ctx, const uint8_t *labels, int nx, int ny, int nz, int labels_on_device,
                        int n_sub, int pad, uint8_t *pack_device);

/* ------------------------------------------------------------------------
 * Learned surrogate of the subimage stiffness (an addition to the paper's
 * method: it replaces the FFT solve of Sec. 4 for subimages a gate accepts,
 * and the FFT solve stays the fallback and the reference for its error).
 * A 3-D CNN maps the one-hot phase labels of an n^3 subimage to its 21
 * stiffness components: four 3x3x3 stride-2 convolutions (8 -> 32 -> 32 ->
 * 64 -> 64 channels, ReLU) and a global mean give 64 features; the window's
 * 8 phase fractions, standardized (hh_net_set_fraction_scaling), are
 * appended, and a linear map takes the 72 features to 21 outputs.  Trained
 * on FFT-solver labels.  Convolutions run on BF16 MFMA with FP32
 * accumulation; parameters are FP32.
 *
 * Inputs of every call: `batch` boxes of box^3 uint8 labels stored back to
 * back; the network reads the n^3 window at (offset, offset, offset) of each
 * box (n = input edge given at creation, offset + n <= box).
 * Outputs are "normalized" (y = (C21 - mean) / scale per component, see
 * hh_net_set_scaling) except hh_net_predict, which returns C21 in GPa.
 * ------------------------------------------------------------------------ */
typedef struct hh_net hh_net;

/* New network for nphase (1..8) phases and input edge n (multiple of 16,
 * <= 256); He-normal weights from `seed`, identity scaling. */
int hh_net_create(hh_ctx *ctx, int nphase, int n, unsigned long long seed, hh_net **net);
void hh_net_destroy(hh_net *net);
long long hh_net_num_params(const hh_net *net);
/* Phase count and input edge of a network. */
int hh_net_info(const hh_net *net, int *nphase, int *n);
/* A network from the file the training pipeline writes (numpy .npz: arrays
 * params <f4 [hh_net_num_params], mean and scale <f8 [21], fmu and fsc <f8
 * [8], n and nphase <i8 scalars; other members are ignored), read on the
 * host with zlib; optional <f8 scalars imu and isc set the interface
 * statistics (hh_net_set_interface_stats).  *net is created on ctx and owned by the caller
 * (hh_net_destroy).  HH_EINVAL for a missing or malformed file, with the
 * reason in hh_last_error(ctx). */
int hh_net_load(hh_ctx *ctx, const char *path, hh_net **net);
/* FP32 parameters (host copies); setting also resets the optimizer state. */
int hh_net_get_params(hh_ctx *ctx, hh_net *net, float *params, long long n);
int hh_net_set_params(hh_ctx *ctx, hh_net *net, const float *params, long long n);
/* Output scaling: C21 = mean + scale * y (scale > 0). */
int hh_net_set_scaling(hh_ctx *ctx, hh_net *net, const double mean[21], const double scale[21]);
int hh_net_get_scaling(const hh_net *net, double mean[21], double scale[21]);
/* Phase-fraction features: feature_c = (f_c - mean[c]) * scale[c] for the
 * fraction f_c of label c in the input window (c = 0..7; default 0 and 1). */
int hh_net_set_fraction_scaling(hh_ctx *ctx, hh_net *net, const double mean[8], const double scale[8]);
int hh_net_get_fraction_scaling(const hh_net *net, double mean[8], double scale[8]);
/* Input-space test of the surrogate gate (hh_hierarchical_surrogate): an
 * item goes to the FFT solver when a label's fraction f_c in this
 * network's input window lies more than z_max feature scales from the
 * mean, |f_c - mean_c| * scale_c > z_max (the fraction scaling above: the
 * training windows' mean and inverse standard deviation), or, for a label
 * whose scale is 0 (its fraction never varied in training), differs from
 * mean_c by at least one voxel.  Default 5; z_max = 0 switches the test
 * off.  HH_EINVAL for a negative or non-finite z_max. */
int hh_net_set_fraction_gate(hh_ctx *ctx, hh_net *net, double z_max);
/* Texture test of the same gate: the interface density d of a window is
 * the fraction of its face-adjacent voxel pairs (along x, y and z, inside
 * the window: 3 n^2 (n - 1) pairs) whose labels differ.  An item goes to
 * the FFT solver when |d - mean| * scale > z_max (the limit above) for this
 * network's input window; mean and scale are the training windows' mean
 * and inverse standard deviation of d.  scale = 0 (the default) switches
 * the test off.  HH_EINVAL unless 0 <= mean <= 1 and scale is finite and
 * >= 0. */
int hh_net_set_interface_stats(hh_ctx *ctx, hh_net *net, double mean, double scale);
int hh_net_get_interface_stats(const hh_net *net, double *mean, double *scale);
/* Normalized outputs y (host, batch x 21). */
int hh_net_forward(hh_ctx *ctx, hh_net *net, const uint8_t *labels, int labels_on_device, int batch, int box,
                   int offset, float *out);
/* Mean squared error against normalized targets (host, batch x 21) and its
 * gradient w.r.t. every parameter (host, hh_net_num_params floats; may be
 * NULL).  Parameters are not changed. */
int hh_net_gradient(hh_ctx *ctx, hh_net *net, const uint8_t *labels, int labels_on_device, int batch, int box,
                    int offset, const float *target, float *loss, float *grad);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on that loss. */
int hh_net_train_step(hh_ctx *ctx, hh_net *net, const uint8_t *labels, int labels_on_device, int batch, int box,
                      int offset, const float *target, int target_on_device, float lr, float *loss);
/* Predicted stiffness C21 in GPa (host, batch x 21). */
int hh_net_predict(hh_ctx *ctx, hh_net *net, const uint8_t *labels, int labels_on_device, int batch, int box,
                   int offset, double *C21);

/*
 * Two-level scheme with the surrogate: the subimage stiffnesses come from
 * the network(s) on every padded box, each network reading the n_sub^3 core
 * or the whole (n_sub + 2 pad)^3 box as its input edge says; a gate sends an
 * item to the FFT solver (the hh_hierarchical path) when the mean prediction
 * is not positive definite, leaves the Voigt-Reuss bracket of the core's
 * phase fractions by more than bound_tol (relative, Mandel norm), when a
 * network's input window has phase fractions or an interface density outside
 * the range the network was trained on (hh_net_set_fraction_gate,
 * hh_net_set_interface_stats), or - with two networks - when the two
 * predictions differ by more than spread_tol (relative).  net_b may be NULL.  fallback: (N/n)^3 flags (may be NULL);
 * C_sub as in hh_hierarchical.  report.items counts subimages,
 * report.voxel_iters the fallback and level-2 solves.
 */
int hh_hierarchical_surrogate(hh_ctx *ctx, const uint8_t *labels, int nx, int ny, int nz, int labels_on_device,
                              const hh_phase *phases, int nphase, int n_sub, int pad, hh_net *net_a,
                              hh_net *net_b, double spread_tol, double bound_tol, const hh_opts *opts,
                              double C_out[36], double *C_sub, int *fallback, hh_report *report);

/*
 * Persistent autotuner cache: reads the tile plans stored in the text file
 * `path` for this GPU architecture and build (lines "hh-plan <arch> <tag>
 * nx ny nz precision aniso bucket z y x"; others are skipped), and appends
 * every plan the context tunes from now on.  A missing file is created by
 * the first tuned shape; an unwritable one only costs tuning time.  Plans
 * change speed, never results (every tile variant gives the same bits).
 * path = NULL stops the appending.
 */
int hh_plan_cache(hh_ctx *ctx, const char *path);

/*
 * Attaches the networks and gate tolerances that hh_hierarchical uses with
 * use_surrogate = 1 (same meaning as in hh_hierarchical_surrogate; net_b may
 * be NULL).  The caller keeps ownership: the networks must stay alive while
 * attached; net_a = NULL detaches.  HH_EINVAL for net_b without net_a or bad
 * tolerances.
 */
int hh_set_surrogate(hh_ctx *ctx, hh_net *net_a, hh_net *net_b, double spread_tol, double bound_tol);

/*
 * Least-squares fit M(n) = M_inf + slope / n of each of the 36 entries over
 * m >= 2 distinct subimage sizes (Sec. 5, eq_fit_power_law).  C: m x 36
 * (row i belongs to n[i]).  Host only.
 */
int hh_richardson(const int *n, const double *C, int m, double C_inf[36], double slope[36]);

/* Bulk and shear moduli of the Voigt isotropic projection of a 6x6
 * stiffness: K = (C11+C22+C33 + 2(C12+C13+C23))/9,
 * G = (C11+C22+C33 - (C12+C13+C23) + 3(C44+C55+C66))/15.  Host only. */
int hh_moduli(const double C[36], double *K, double *G);

/* The arithmetic-mean comparator of Sec. 5 (AM): the mean over m subimages
 * of the Voigt bulk and shear moduli (as hh_moduli) of their stiffnesses.
 * C_sub: m x 21 upper-triangle components, as hh_hierarchical writes them.
 * Host only; HH_EINVAL for m < 1 or NULL pointers. */
int hh_mean_moduli(const double *C_sub, long long m, double *K, double *G);

#ifdef __cplusplus
}
#endif

#endif /* HH_H */
