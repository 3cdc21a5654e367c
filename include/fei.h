/* fei.h -- batched finite-element element-matrix integration on MI355X (gfx950).
 *
 * The library computes, for every simplex e of a mesh, the dense element
 * matrix of a bilinear form as the tensor contraction of the paper
 * "Finite Element Integration on GPUs" (Knepley & Terrel), Sec. 3, eq. 1:
 *
 *     A_e = G_e : K
 *
 * K (the reference or "analytic" tensor, eq. 7) depends only on the form and
 * the reference simplex and is precomputed once per form (Sec. 3.1, last
 * paragraph).  G_e (the geometric tensor, eq. 8) is formed inside the kernels
 * from the element's vertex coordinates: the Jacobian J, its inverse and
 * |det J|, and, for elasticity, the element's Lame coefficients.
 *
 * Forms (affine simplices, dim = 2 or 3):
 *   FEI_LAPLACE_P1  A_ij = int grad phi_i . grad phi_j           (Sec. 3, eqs. 2-8)
 *   FEI_ELASTIC_P1  A_IJ = int 2 mu eps(Phi_I):eps(Phi_J)
 *                             + lambda div Phi_I div Phi_J        (Sec. 3, eqs. 9-15,
 *                   with per-element Lame mu, lambda; mu = 1/2, lambda = 0 is the
 *                   form of eq. 24)
 *   FEI_LAPLACE_P2  as FEI_LAPLACE_P1 with the quadratic Lagrange basis
 *
 * Conventions shared by every entry point:
 *   - Reference simplex: vertex 0 at the origin, vertex m+1 at e_m.  The
 *     element's vertex conn[e][0] is the origin of J:
 *     J[alpha][m] = x_{conn[e][m+1]}[alpha] - x_{conn[e][0]}[alpha].
 *   - Element matrix size n: P1 Laplacian dim+1; P1 elasticity dim*(dim+1);
 *     P2 Laplacian (dim+1)(dim+2)/2.  Vector DOFs are node-major, I = dim*a + c.
 *     P2 DOFs: the dim+1 vertices, then edges (0,1),(0,2),..,(0,dim),(1,2),..
 *   - Output A is row-major [E][n][n] FP32 (symmetric, so equally column-major).
 *   - All mesh, coefficient and output arrays are DEVICE memory owned by the
 *     caller.  Entry points that take a stream enqueue work on it and return
 *     without synchronising; outputs are valid once the stream reaches them.
 *   - |det J| is used for the volume, so either orientation integrates
 *     correctly.  An element with det J == 0 yields Inf/NaN entries (IEEE) and
 *     is counted (see fei_options.counters); the call still succeeds.
 *
 * Errors: every int-returning call returns FEI_OK (0) or a negative status.
 * On error nothing is enqueued and no output is written.  fei_last_error()
 * returns a thread-local message for the last failing call.  No entry point
 * throws, aborts or exits.
 */
#ifndef FEI_H
#define FEI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEI_ABI_VERSION 2

enum fei_status {
    FEI_OK = 0,
    FEI_EINVAL = -1,      /* bad argument: null/misaligned pointer, bad form, dim, dtype, size */
    FEI_EDEVICE = -2,     /* a HIP call failed; message in fei_last_error() */
    FEI_ENOMEM = -3,      /* host or device allocation failed (plans only) */
    FEI_EUNSUPPORTED = -4 /* valid request the library has no kernel for */
};

enum fei_form {
    FEI_LAPLACE_P1 = 1,
    FEI_ELASTIC_P1 = 2,
    FEI_LAPLACE_P2 = 3
};

enum fei_dtype { FEI_F32 = 0, FEI_F64 = 1 };

/* Arithmetic of the G:K contraction.  Geometry (J, J^-1, |J|, G) is always
 * FP32, or FP64 for FP64 coordinates and for elements flagged by the quality
 * test below.
 *   FEI_PREC_FP32    FP32 fused multiply-adds.
 *   FEI_PREC_FP16X2  MFMA: G split into FP16 hi + lo after per-element
 *                    power-of-two scaling; K is exact in FP16; FP32 accumulate.
 *   FEI_PREC_BF16X2  MFMA: G split into BF16 hi + lo (about 16 bits).
 *   FEI_PREC_BF16X3  MFMA: G split into three BF16 terms (about 24 bits).   */
enum fei_precision {
    FEI_PREC_FP32 = 0,
    FEI_PREC_FP16X2 = 1,
    FEI_PREC_BF16X2 = 2,
    FEI_PREC_BF16X3 = 3
};

/* Layouts of the reference tensor returned by fei_reference_tensor.
 *   FEI_LAYOUT_BLOCK   K[i][j][mu][nu] = int_ref dphi_i/dxi_mu dphi_j/dxi_nu
 *                      (eq. 7), [nb][nb][dim][dim] over the SCALAR basis of
 *                      the form (for elasticity the vector element's tensor
 *                      is this one times delta_cc' delta_dd', eq. 14).
 *   FEI_LAYOUT_FOLDED  the integer-valued matrix Kf[g][n*n] the kernels use:
 *                      A_e = sum_g Gf_e[g] Kf[g][:], where Gf_e holds the g
 *                      unique entries of the symmetric geometric tensor times
 *                      fei_reference_scale(form, dim).                        */
enum fei_layout { FEI_LAYOUT_BLOCK = 0, FEI_LAYOUT_FOLDED = 1 };

typedef struct fei_mesh {
    int32_t dim;            /* 2 or 3 */
    int32_t coord_dtype;    /* FEI_F32 or FEI_F64 */
    int64_t n_vertices;     /* >= 1 unless n_elements == 0 */
    int64_t n_elements;     /* 0 <= n_elements <= 2^32 - 256 */
    const void *x;          /* device [n_vertices] coordinates (SoA) */
    const void *y;
    const void *z;          /* NULL when dim == 2 */
    const int32_t *conn;    /* device [n_elements][dim+1], 0 <= v < n_vertices */
} fei_mesh;

typedef struct fei_options {
    int32_t precision;      /* enum fei_precision */
    float tau;              /* quality threshold: an element whose
                               kappa = |J|_F |adj J|_F / |det J| (computed in
                               FP32) exceeds tau takes the FP64 geometry path.
                               <= 0 forces FP64 for every element; +Inf never. */
    int32_t *counters;      /* optional device int32[2], accumulated (+=):
                               [0] elements that took the FP64 path,
                               [1] elements with det J == 0.  NULL: none. */
    int32_t store_rows;     /* how element matrices leave the kernels (a tuning
                               knob, the paper's interleaved stores, Sec. 4.3):
                               0 = the tuned default; -1 = every lane stores
                               its own rows; R > 0 = the wave stages R rows of
                               all its elements' matrices in LDS and stores
                               them with contiguous 16-byte pieces; R = n
                               stages whole matrices, which leave as one
                               contiguous run per chunk of elements (the
                               forward's default; the adjoint reads dA in R-row
                               chunks the same way).  R must divide n with
                               R*n a multiple of 4 (the forward also takes
                               R = n for any n: 3x3 matrices are staged
                               packed), and for the adjoint also R*n <= 48
                               or R = n (whole matrices, staged 64 or 32
                               elements at a time); FEI_EUNSUPPORTED
                               otherwise. */
    int32_t block_elements; /* forward, FP32 contraction, default staging:
                               elements per workgroup (the paper's element
                               batch size, Sec. 4), 64, 128, 256 or 512;
                               0 = the tune table's choice for this form, dim,
                               precision and size (fei_tune_forward), else 256.
                               FEI_EUNSUPPORTED for other precisions or
                               staging with a value other than 0 or 256. */
    int32_t reserved[3];    /* must be zero */
} fei_options;

/* Version of this ABI (FEI_ABI_VERSION). */
int fei_abi_version(void);

/* Static description of a status code. */
const char *fei_status_str(int status);

/* Thread-local message describing the last failing call on this thread. */
const char *fei_last_error(void);

/* Fills *opt with defaults: FP32, tau = 100, no counters, tuned staging. */
int fei_options_default(fei_options *opt);

/* Element matrix size n for (form, dim), or FEI_EINVAL. */
int fei_local_size(int form, int dim);

/* The reference tensor K of (form, dim) in the given layout, into HOST memory.
 * With K == NULL only *len (number of floats) is written.  For the folded
 * layout *g_out (if not NULL) receives g.  Host-only: needs no device.
 * Sec. 3, eq. 7 (block layout) and eq. 1 (the contraction the folded layout
 * serves).                                                                   */
int fei_reference_tensor(int form, int dim, int layout, float *K, int64_t *len,
                         int32_t *g_out);

/* Scale s with Gf = s * |det J| * (unique entries of J^-1 J^-T [elasticity:
 * of its Lame analogue]); the folded K is K_block / (s * ... ) made integral. */
double fei_reference_scale(int form, int dim);

/* Forward: A[e] = G_e : K for every element (Sec. 3, eqs. 1, 6-8, 14-15).
 *   m        mesh (host struct, device arrays)
 *   form     enum fei_form
 *   mu, lam  device [E] FP32 Lame coefficients for FEI_ELASTIC_P1, NULL otherwise
 *   A        device [E][n][n] FP32, 16-byte aligned, overwritten
 *   opt      NULL for defaults
 *   stream   hipStream_t (NULL: the null stream)                            */
int fei_integrate(const fei_mesh *m, int form, const float *mu, const float *lam,
                  float *A, const fei_options *opt, void *stream);

/* The Laplacian with a P1 coefficient w (Sec. 3.1, eqs. 20-23):
 *   A[e]_ij = int_e w grad phi_i . grad phi_j,   w = sum_k w_k phi_k (P1),
 * computed as sum_k w_k G^{mu nu} K^{ijk}_{mu nu} with the arity-3 reference
 * tensor K^{ijk} (fei_reference_tensor_coefficient) and G of eq. 8.
 *   form     FEI_LAPLACE_P1 or FEI_LAPLACE_P2 (FEI_EUNSUPPORTED otherwise)
 *   w        device [n_vertices] FP32: the coefficient's value at each vertex
 *   A        device [E][n][n] FP32, 16-byte aligned, overwritten
 *   opt      precision must be FEI_PREC_FP32; tau, counters and store_rows
 *            (0, -1, n, or 2 where 2n is a multiple of 4) as for fei_integrate
 * Asynchronous on `stream`.                                                 */
int fei_integrate_coefficient(const fei_mesh *m, int form, const float *w, float *A,
                              const fei_options *opt, void *stream);

/* K^{ijk}_{mu nu} = int_ref dphi_i/dxi_mu phi_k dphi_j/dxi_nu (k over the P1
 * coefficient's vertices) of FEI_LAPLACE_P1 / FEI_LAPLACE_P2, into HOST memory
 * as [nb][nb][dim+1][dim][dim]; with K == NULL only *len is written.        */
int fei_reference_tensor_coefficient(int form, int dim, float *K, int64_t *len);

/* The isoparametric P2 Laplacian on elements with quadratic geometry (Sec.
 * 3.1, eqs. 16-19): the geometry map and the solution basis are the P2 basis
 * of the element's nodes; following the paper the inverse Jacobian is
 * projected into a finite element space -- the vertex functions, by its
 * values at the vertices -- and |J| is taken out of the integral as one
 * constant, |det J| at the barycenter, so that
 *   A_ij = G^{(k mu),(l nu)} K^{ijkl}_{mu nu},
 *   G^{(k mu),(l nu)} = J^-1_{mu alpha,k} J^-1_{nu alpha,l} |J_c|,
 * with the arity-4 reference tensor K^{ijkl}_{mu nu} = int_ref lambda_k
 * dphi_i/dxi_mu lambda_l dphi_j/dxi_nu (exact, built with the library).
 * Straight edges (edge nodes at the midpoints) give FEI_LAPLACE_P2 exactly.
 *   m        dim 2 or 3, FP32 coordinates of all nodes (n_vertices = nodes),
 *            conn device [E][nb] (nb = 6 or 10): the vertices, then the edge
 *            nodes in the P2 order (0,1),(0,2),..
 *   A        device [E][nb][nb] FP32, 16-byte aligned, overwritten
 *   opt      precision FP32, store_rows 0; tau (applied to the Jacobians at
 *            the vertices and the barycenter) and counters as for fei_integrate
 * Asynchronous on `stream`.                                                 */
int fei_integrate_iso(const fei_mesh *m, float *A, const fei_options *opt, void *stream);

/* Adjoint of fei_integrate for L = sum_e <dA_e, A_e> (the reverse of the
 * chain A_e <- G_e <- (J^-1, |J|) <- vertex coordinates, Lame coefficients),
 * with G recomputed from the mesh rather than stored.
 *   dA          device [E][n][n] FP32, any (not necessarily symmetric) values
 *   dx, dy, dz  device [n_vertices] FP32: dL/dx is ADDED (+=) by FP32 atomics;
 *               dz is NULL in 2D.  The caller zeroes them first if needed.
 *               Summation order is not deterministic.
 *   dmu, dlam   device [E] FP32, overwritten (FEI_ELASTIC_P1 only; NULL skips)
 *   opt         precision: FEI_PREC_FP32 (default), or FEI_PREC_FP16X2 /
 *               BF16X2 / BF16X3: the fold of dA with K (the contraction of
 *               eq. 1 in reverse, U_g = sum_ij Kf[g][ij] dA_ij) runs on the
 *               matrix cores with dA split into two or three 16-bit terms
 *               (FP16 with a power-of-two scale per element); K is exact in
 *               both formats, so only dA carries split error (FP16x2 and
 *               BF16x3 about FP32's, BF16x2 about 2^-16 of the largest
 *               entry).  These need FP32 coordinates, store_rows 0 or n, and
 *               n*n a multiple of 4 (FEI_EUNSUPPORTED for the 3 x 3 matrices
 *               of the 2D P1 Laplacian).  Elements flagged by the quality
 *               test fold in FP64 in every precision.                        */
int fei_integrate_adjoint(const fei_mesh *m, int form, const float *mu,
                          const float *lam, const float *dA, float *dx, float *dy,
                          float *dz, float *dmu, float *dlam,
                          const fei_options *opt, void *stream);

/* The adjoint of fei_integrate_adjoint with vertex gradients summed in an
 * order fixed by the mesh, so every call gives the same bits (FP32
 * coordinates only; store_rows must be 0).  Same arguments, same meaning:
 * dx, dy, dz are accumulated (+=) -- without atomics, by one read-modify-write
 * per vertex -- and dmu, dlam are overwritten.  Steps, all on `stream`: the
 * vertex-to-element incidence of the mesh (CSR, built on the device), J-bar
 * per element (the reverse of eqs. 5 and 8 per element), then each vertex
 * sums the contributions of its elements in increasing element order.  The
 * workspace, 4 (N_v + 1) + 4 N_v + 4 (dim + 1) E + 4 dim^2 E bytes (each part
 * rounded up to 256), is taken with hipMallocAsync and released with
 * hipFreeAsync on the stream.  FEI_ENOMEM if that allocation fails.        */
int fei_integrate_adjoint_det(const fei_mesh *m, int form, const float *mu,
                              const float *lam, const float *dA, float *dx, float *dy,
                              float *dz, float *dmu, float *dlam,
                              const fei_options *opt, void *stream);

/* fei_integrate_adjoint_det for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, same results (bit for bit), but the workspace
 * lives in a fixed device array of the library, FEI_NOALLOC_SCRATCH_BYTES
 * bytes, one per device, held from its first use until the process ends; the
 * call allocates and frees nothing.  The workspace of a mesh is
 * 4 (N_v + 1) + 4 N_v + 4 (dim + 1) E + 4 dim^2 E bytes (each part rounded up
 * to 256; the 3D elasticity workload of 1,572,864 tets and 290,353 vertices
 * needs 84 MB): FEI_EINVAL if that exceeds FEI_NOALLOC_SCRATCH_BYTES.
 * `stream` must belong to the current device.  Every call on one device
 * shares that device's array, which keeps the last call's contents: calls
 * whose work overlaps on one device (other streams, other threads) race and
 * must be ordered by the caller.                                            */
#define FEI_NOALLOC_SCRATCH_BYTES (96u * 1024u * 1024u)
int fei_integrate_adjoint_det_noalloc(const fei_mesh *m, int form, const float *mu,
                                      const float *lam, const float *dA, float *dx, float *dy,
                                      float *dz, float *dmu, float *dlam,
                                      const fei_options *opt, void *stream);

/* ---- tuning ------------------------------------------------------------------
 * A process-wide tune table maps (form, dim, precision, coordinate type, size
 * bucket = floor(log2 E)) to the forward's elements per workgroup and output
 * staging; fei_integrate consults it when opt->block_elements and
 * opt->store_rows are both 0.  If the environment variable FEI_TUNE_FILE names
 * a file, the table is loaded from it on first use.                          */
typedef struct fei_tune_result {
    int32_t block_elements;     /* chosen elements per workgroup */
    int32_t store_rows;         /* chosen staging (0: the form's default) */
    float ms;                   /* its mean time per launch */
    int32_t candidates;         /* configurations timed */
} fei_tune_result;

/* Times the forward's candidate configurations (elements per workgroup 64,
 * 128, 256, 512 and the staging variants for FP32; staged or direct stores
 * for the MFMA precisions) on the caller's data -- A is written by every
 * trial -- records the fastest in the tune table and returns it in *out (if
 * not NULL).  Arguments as for fei_integrate (opt->block_elements and
 * opt->store_rows are ignored).  Synchronizes `stream`.                     */
int fei_tune_forward(const fei_mesh *m, int form, const float *mu, const float *lam, float *A,
                     const fei_options *opt, void *stream, fei_tune_result *out);
/* The table's entry for a call, if any: returns 1 and fills *out when present,
 * 0 when not.  Host-only.                                                    */
int fei_tune_lookup(int form, int dim, int precision, int coord_dtype, int64_t n_elements,
                    fei_tune_result *out);
/* Writes the table as JSON lines ({"arch": .., "form": .., "dim": .., "precision": ..,
 * "coord": .., "ebucket": .., "block_elements": .., "store_rows": .., "ms": ..}),
 * or reads such a file and merges its entries (entries of another GPU
 * architecture are skipped when a device is present).  Host-only.          */
int fei_tune_save(const char *path);
int fei_tune_load(const char *path);
/* Empties the table.                                                         */
int fei_tune_clear(void);

/* Checks conn against n_vertices on the device and returns the number of
 * out-of-range entries in *n_bad.  Synchronises the stream.                 */
int fei_validate_mesh(const fei_mesh *m, int64_t *n_bad, void *stream);

/* ---- heterogeneous batches ------------------------------------------------
 * Many meshes and forms integrated by one launch of a HIP graph (the paper's
 * element batches, Sec. 4, applied across meshes).  Items are ordered
 * heaviest first (algorithmic bytes) and cut into 256-element tiles.  Four
 * graph shapes exist (fei_batch_config.mode):
 *   0  one persistent kernel for all forms: workgroups take tiles from a
 *      work counter (reset by a kernel node) until none are left;
 *   1  one kernel per (form, dim) group, the groups captured as concurrent
 *      branches of the graph (each kernel has the registers and LDS of its
 *      own form only);
 *   2  the single-mesh kernels of fei_integrate / fei_integrate_adjoint, one
 *      launch per item, the items of a group in turn on the group's branch;
 *   3  the kernels of mode 1, the groups one after another on one stream
 *      (each has the whole GPU while it runs).
 * fei_batch_tune times candidate configurations on the caller's data and
 * rebuilds the graph with the fastest.
 * The plan owns its descriptor tables, work counter, streams and graphs, and
 * for the adjoint's vertex gather its incidence and J-bar buffers (allocated
 * by fei_batch_create, fei_batch_tune or fei_batch_set_config, released by
 * fei_batch_destroy); every pointer in the items is caller memory that must
 * outlive the plan.  Only FP32 coordinates are accepted in batches.        */
typedef struct fei_batch_item {
    fei_mesh mesh;
    int32_t form;
    int32_t pad_;
    const float *mu, *lam;  /* elasticity only */
    float *A;               /* forward output [E][n][n] */
    const float *dA;        /* adjoint input; NULL leaves the item out of the adjoint */
    float *dx, *dy, *dz;    /* adjoint vertex gradients (accumulated) */
    float *dmu, *dlam;      /* adjoint coefficient gradients (overwritten, may be NULL) */
} fei_batch_item;

typedef struct fei_batch_config {
    int32_t mode;           /* 0: persistent multi-form kernel, 1: per-group kernels
                               on concurrent branches, 2: single-mesh kernels per
                               item, 3: per-group kernels in sequence */
    int32_t variant;        /* modes 0, 1, 3: output staging, 0 wide, 1 narrow */
    int32_t workgroups;     /* mode 0: persistent workgroups launched */
    int32_t tiles_per_pop;  /* mode 0: tiles taken from the counter per atomic */
    float ms;               /* measured time of this configuration (0: not tuned) */
    int32_t gather;         /* adjoint only.  0: vertex gradients by a wave-level
                               merge, then global FP32 atomics (they execute at
                               the memory side); 1: J-bar per element into a
                               plan buffer, then each vertex sums its
                               elements' terms in an order fixed by the mesh --
                               no atomics (unless two items share gradient
                               arrays), and every run of the graph gives the
                               same bits.  Setting 1 first builds the plan's
                               vertex-to-element incidence from the items'
                               connectivity (device-synchronizing; the plan
                               then holds 4 (N_v + 1) + 4 (d + 1) E + 4 d^2 E
                               bytes per item). */
    int32_t reserved[2];    /* must be zero */
} fei_batch_config;

typedef struct fei_batch fei_batch;

/* Validates every item, builds the plan and its graphs with the default
 * configuration (mode 1, variant 0).  opt: precision and tau (NULL: defaults);
 * the adjoint is FP32.  Does not touch the items' data.                     */
int fei_batch_create(const fei_batch_item *items, int n_items, const fei_options *opt,
                     fei_batch **out);
/* One graph launch on `stream`: every item's forward (or adjoint).          */
int fei_batch_run(fei_batch *b, void *stream);
int fei_batch_run_adjoint(fei_batch *b, void *stream);
/* Times the candidate configurations of the forward (adjoint = 0) or adjoint
 * (adjoint = 1, both gather settings: builds the vertex incidence first) graph
 * on `stream`, each as an instantiated graph launched as fei_batch_run does
 * (one warm-up, the median of three) -- running them, so outputs are written,
 * and for the adjoint dx/dy/dz receive one accumulation per trial -- then
 * rebuilds that graph with the fastest.  *chosen (if not NULL) receives it.  */
int fei_batch_tune(fei_batch *b, int adjoint, void *stream, fei_batch_config *chosen);
int fei_batch_get_config(const fei_batch *b, int adjoint, fei_batch_config *out);
/* Rebuilds the forward/adjoint graph with a given configuration (for example
 * one returned by an earlier fei_batch_tune).  mode 0 needs workgroups >= 1
 * and tiles_per_pop >= 1; variant and gather are 0 or 1 (gather = 1 only for
 * the adjoint); reserved must be zero.                                      */
int fei_batch_set_config(fei_batch *b, int adjoint, const fei_batch_config *cfg);
/* Copies the vertex-to-element incidence the plan built for item `item` (an
 * index into the list given to fei_batch_create) for the adjoint's vertex
 * gather, so callers and tests can inspect it.  The incidence is CSR over
 * vertices: ptr[v] .. ptr[v+1] index inc, whose entries are e * (dim + 1) + a
 * (element e, local vertex a) in increasing order.
 *   ptr  device int32[n_vertices + 1], written
 *   inc  device int32[(dim + 1) * n_elements], written
 * Asynchronous on `stream`.  FEI_EINVAL if the plan has not built its vertex
 * gather (fei_batch_tune with adjoint = 1, or fei_batch_set_config with
 * gather = 1) or the item is not part of the adjoint (no dA or no elements). */
int fei_batch_copy_incidence(const fei_batch *b, int item, int32_t *ptr, int32_t *inc,
                             void *stream);
int fei_batch_destroy(fei_batch *b);

/* ---- fused global assembly -------------------------------------------------
 * The global matrix K = sum_e P_e^T A_e P_e of a P1 form (the global portion of
 * the computation that element integration feeds, Sec. 1), with each A_e
 * integrated on the fly (Sec. 3, eq. 1) and summed into K's values without
 * ever being stored.  K is CSR over vertices with NC x NC blocks (NC = 1 for
 * FEI_LAPLACE_P1, dim for FEI_ELASTIC_P1; block (i, j) entry (c, d) is the
 * coefficient of DOF dim * j + d in row dim * i + c, the node-major DOF order
 * of the element matrices).  Row i stores every vertex that shares an element
 * with i, in increasing order, even where the sum is zero.
 *
 * A plan holds the pattern and the vertex-to-element incidence the kernel
 * walks, each row's incidences ordered in steps of four whose elements share
 * no vertex but the row's (so a step's blocks are added without conflicts),
 * with the slots of each incidence's element vertices in the row (4 bytes
 * per entry); it is built once per connectivity and serves any coordinates
 * and coefficients on that connectivity. */
typedef struct fei_assembly fei_assembly;

/* Builds the plan of mesh m (its connectivity; coordinates are not read).
 * Device-synchronizing: the connectivity is copied to the host, checked
 * (FEI_EINVAL for an entry outside [0, n_vertices)) and the pattern built
 * there.  FEI_EUNSUPPORTED for P2 forms and for a vertex with more than 256
 * neighbours.  The plan owns its device arrays, released by
 * fei_assembly_destroy.                                                     */
int fei_assembly_create(const fei_mesh *m, int form, fei_assembly **out);
/* Rows (= n_vertices), stored blocks, and the block side NC.                */
int fei_assembly_info(const fei_assembly *a, int64_t *n_rows, int64_t *nnz, int32_t *block);
/* Copies the pattern into device arrays rowptr [n_rows + 1] and colidx [nnz]
 * (int32), asynchronously on `stream`.                                      */
int fei_assembly_copy_pattern(const fei_assembly *a, int32_t *rowptr, int32_t *colidx,
                              void *stream);
/* The incidence schedule the kernel walks: *n_entries receives its length;
 * with ptr and inc non-NULL, copies ptr [n_rows + 1] and inc [n_entries]
 * (device int32, asynchronously on `stream`).  Row v's entries are
 * inc[ptr[v] .. ptr[v + 1]), in steps of 4 (ptr[v + 1] - ptr[v] is a
 * multiple of 4); an entry is e * (dim + 1) + a (element e, local vertex a of
 * v) or -1 (padding).  The elements of one step share no vertex but v, and
 * every incidence of v appears once.                                        */
int fei_assembly_copy_schedule(const fei_assembly *a, int64_t *n_entries, int32_t *ptr,
                               int32_t *inc, void *stream);
/* values [nnz][NC][NC] FP32 (device, overwritten) = K of mesh m, which must
 * have the dimension, vertex and element counts of the plan's mesh and the
 * same connectivity (not re-checked: the kernel trusts the plan); FP32
 * coordinates; mu, lam as for fei_integrate.  opt: precision must be FP32;
 * tau and counters act as in fei_integrate (each element counted once).
 * Every element is integrated once per vertex (by the wave that owns that
 * vertex's row), so each block's sum is formed in LDS and written once.
 * Asynchronous on `stream`.                                                 */
int fei_assemble(const fei_assembly *a, const fei_mesh *m, const float *mu, const float *lam,
                 float *values, const fei_options *opt, void *stream);
int fei_assembly_destroy(fei_assembly *a);

/* ---- form front end ---------------------------------------------------------
 * Bilinear forms of Lagrange elements described at run time (the forms a form
 * language describes, Sec. 3.2), integrated by the same contraction (Sec. 3,
 * eq. 1) with a reference tensor built a priori (Sec. 3.1):
 *
 *   A_{(i,c),(j,d)} = int_e sum_{a,b} C[(a,c),(b,d)] D_a phi_i D_b phi_j
 *                   = sum_{p,q} G_{(p,c),(q,d)} Khat_ij^{pq}
 *
 * D_0 = the value, D_{1+alpha} = d/dx_alpha; C = W_0 + sum_k coef_k(e) W_k with
 * per-element coefficients; Khat_ij^{pq} = int_ref Dhat_p phi_i Dhat_q phi_j
 * over values and reference derivatives (eq. 7 extended to values), computed
 * exactly; G = |det J| That^T C That with That the map from physical to
 * reference derivatives (J^-1, eq. 8).  DOFs node-major, I = ncomp * i + c;
 * the P2 basis and its DOF order as in FEI_LAPLACE_P2.                     */
typedef struct fei_weak_form fei_weak_form;

/* Compiles a form: dim 2 or 3, degree 1 or 2, ncomp 1 (scalar) or dim
 * (vector), 0 <= n_coef <= 4 per-element coefficients, and the operator
 * tables W [n_coef + 1][m][m] (HOST, m = (dim + 1) * ncomp, index a * ncomp + c,
 * row = the test function's operator) -- the weak-form description.  Builds
 * Khat and uploads W and Khat (the plan owns them; FEI_ENOMEM if that fails).
 * A form whose tables are all symmetric is integrated as symmetric.          */
int fei_form_create(int dim, int degree, int ncomp, int n_coef, const double *W,
                    fei_weak_form **out);
/* Element matrix size n, whether the form is symmetric, and n_coef.          */
int fei_form_info(const fei_weak_form *f, int32_t *n, int32_t *symmetric, int32_t *n_coef);
/* Khat [nb][nb][dim + 1][dim + 1] of the degree-`degree` scalar Lagrange basis
 * (double, HOST, the exact rationals rounded once); with K == NULL only *len
 * is written.  Host-only: needs no device.                                  */
int fei_form_reference_tensor(int dim, int degree, double *K, int64_t *len);
/* A[e] (device [E][n][n] FP32, 16-byte aligned, overwritten) for every element
 * of m (FP32 coordinates, m->dim == the form's dim); coef device [n_coef][E]
 * FP32 (NULL when n_coef == 0).  opt: precision FP32, store_rows 0; tau and
 * counters as for fei_integrate.  Asynchronous on `stream`.                 */
int fei_form_integrate(const fei_weak_form *f, const fei_mesh *m, const float *coef, float *A,
                       const fei_options *opt, void *stream);
/* Generates and compiles a kernel for this form (what a form compiler does,
 * Sec. 3.2): the generic kernel's steps with W and Khat as compile-time
 * constants, so their zero entries and the unused coefficients drop out;
 * later fei_form_integrate calls launch it (same results up to the sign of
 * zero: the dropped terms are exact zeros).  Runs the HIP compiler
 * (FEI_HIPCC, else $ROCM_PATH/bin/hipcc, else /opt/rocm/bin/hipcc) on the
 * current device's architecture with the kernel headers next to this library,
 * and caches the code object in FEI_JIT_DIR (default $TMPDIR/fei_jit_<uid>)
 * under a hash of the source, so a form already compiled is only loaded.
 * Synchronous, seconds when compiling.  FEI_EUNSUPPORTED when the compiler or
 * the headers are missing, FEI_EDEVICE when compiling or loading fails (the
 * form keeps its generic kernel).                                          */
int fei_form_compile(fei_weak_form *f);
/* 1 when fei_form_compile has given the form its own kernel, else 0.         */
int fei_form_is_compiled(const fei_weak_form *f);
int fei_form_destroy(fei_weak_form *f);

#ifdef __cplusplus
}
#endif

#endif /* FEI_H */
