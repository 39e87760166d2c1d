/*
 * fem.h -- C ABI of libfem: element stiffness-matrix and load-vector integration for
 * tensor-product Lagrange hexahedra of degree p = 1..7 on one AMD Instinct MI355X (gfx950).
 *
 * The operation is the element-level numerical integration of Banas, Plaszewski and Maciol,
 * "Numerical integration on GPUs for higher order finite elements": Algorithm 1 and
 * Algorithm 2 of section 2 (loop over quadrature points; per point the Jacobian, its
 * determinant and inverse, the physical derivatives psi, the point coefficients c^Q, then an
 * update of every entry of A^e), with the element entry of eq. (sum_int) of section 5.1,
 * specialised to one scalar unknown and the convection-diffusion-reaction form
 *
 *   A[i][j] = sum_q w_q detJ_q [ sum_kl K_kl d_k phi_i d_l phi_j
 *                                + phi_i sum_k b_k d_k phi_j + c phi_i phi_j ]
 *   b[i]    = sum_q w_q detJ_q f phi_i
 *
 * Element conventions. Reference cube [-1,1]^3. Vertex v = v1 + 2 v2 + 4 v3 of an element sits
 * at xi = (2v1-1, 2v2-1, 2v3-1); the geometry is the trilinear map of the 8 vertices. Shape
 * functions are tensor products of the 1-D Lagrange polynomials on the p+1 Gauss-Lobatto-
 * Legendre nodes, node i = a + n b + n^2 c with n = p+1 and Ns = n^3. The quadrature is the
 * (p+1)^3-point Gauss-Legendre rule. J[a][b] = dx_a/dxi_b; physical gradients are J^{-T}
 * times reference gradients. Row i of A is the test function, column j the trial function.
 *
 * Memory. Every array pointer is a DEVICE pointer owned by the caller, unless marked HOST.
 * Nothing is allocated or freed by fem_integrate; fem_init allocates the library's constant
 * tables once per process. Calls enqueue work on `stream` (a hipStream_t; NULL = the null
 * stream) and return without synchronising.
 *
 * Errors. Every function returns a fem_status. Argument errors are detected on the host before
 * anything is enqueued; HIP launch errors map to FEM_EHIP. Data errors (detJ <= 0 at some
 * quadrature point, non-finite values) are counted asynchronously into coeffs->status; such
 * elements are still integrated, with the signed detJ.
 */
#ifndef FEM_H
#define FEM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEM_ABI_VERSION 4

typedef enum {
    FEM_OK = 0,
    FEM_EINVAL = -1,     /* a null pointer, a negative count or an unknown enum value */
    FEM_EDEGREE = -2,    /* p outside 1..7 (or p == 0 without a degree array) */
    FEM_ENOTINIT = -3,   /* fem_init has not succeeded in this process */
    FEM_ENOMEM = -4,     /* fem_init could not allocate its tables */
    FEM_EHIP = -5,       /* a HIP runtime call or kernel launch failed */
    FEM_ECONFIG = -6,    /* no compiled kernel configuration for the request */
    FEM_EWORKSPACE = -7, /* workspace missing or smaller than fem_workspace_bytes() */
    FEM_ETOOBIG = -8     /* fem_integrate_noalloc: more elements than its static scratch holds */
} fem_status;

/* Arithmetic of the contraction A = B^T blockdiag(D_q) B. The Jacobian, its determinant and
 * inverse are computed in FP64 on every path; the load vector is accumulated in FP64.
 *   FEM_FP64        FP64 MFMA, FP64 output
 *   FEM_FP32        FP32 MFMA, FP32 output
 *   FEM_BF16        one BF16 MFMA product per term, FP32 accumulation, FP32 output
 *   FEM_SPLIT_BF16  x = hi + lo in BF16 on both operands; hi*hi + hi*lo + lo*hi, FP32 acc.
 *   FEM_SPLIT_FP16  the same three products in FP16 with exact power-of-two scaling
 */
typedef enum {
    FEM_FP64 = 0,
    FEM_FP32 = 1,
    FEM_BF16 = 2,
    FEM_SPLIT_BF16 = 3,
    FEM_SPLIT_FP16 = 4
} fem_precision;

/* How the coefficients are given (section 2: c per element, or c^Q per quadrature point).
 *   FEM_COEF_ELEMENT  elem[e][14] = K (3x3 row-major), b (3), c, f; constant on the element
 *   FEM_COEF_FIELD    elem[e][10] = Q (3x3 row-major), f; plus `field`, 7 fields x 5 modes x
 *                     (a, k1, k2, k3, theta) = 175 doubles. Field s at x is
 *                     g_s(x) = sum_m a_sm sin(2 pi (k_sm . x) + theta_sm) and at each
 *                     quadrature point x_q: K = Q diag(10^g0, 10^g1, 10^g2) Q^T,
 *                     b = (g3, g4, g5), c = (1 + g6) / 2; f stays per element.
 *   FEM_COEF_ELASTIC  the vector model problem of section 5.1, linear elastostatics with the
 *                     isotropic tensor c_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk)
 *                     of each element's Young modulus E and Poisson ratio nu:
 *                     elem[e][5] = E, nu, f1, f2, f3 (body force). Uniform p only. The
 *                     element matrix is the 3 x 3 block matrix of Ns x Ns blocks
 *                     A[(i,s)][(k,r)] = sum_q c_ijkl d_l phi_r d_j phi_s w_q detJ_q (eq.
 *                     (sum_int)), stored out_A[e][i][k][s][r]; out_b[e][i][s] =
 *                     sum_q f_i phi_s w_q detJ_q. Both are 9 (3) times the scalar sizes.
 *                     The tensor's major symmetry makes block (k, i) the transpose of block
 *                     (i, k); for most degrees the library integrates the blocks with i <= k
 *                     and writes the others as transposed copies (equal up to rounding to
 *                     integrating them). */
typedef enum { FEM_COEF_ELEMENT = 0, FEM_COEF_FIELD = 1, FEM_COEF_ELASTIC = 2 } fem_coef_mode;

/* Per-call description of the coefficients and of optional mixed-degree data. HOST struct,
 * read during the call only; the pointers inside are DEVICE pointers. */
typedef struct fem_coeffs {
    int32_t precision;       /* fem_precision; FEM_FP64 -> out_A/out_b are double, else float */
    int32_t mode;            /* fem_coef_mode */
    const double *elem;      /* [nel][14], [nel][10] or [nel][5] FP64 records, see fem_coef_mode */
    const double *field;     /* [175] FP64, FIELD mode only, else ignored */
    const int8_t *degree;    /* [nel] per-element degree 1..7 when p == 0, else ignored */
    const int64_t *a_off;    /* [nel+1] element offsets (in entries) into out_A when p == 0 */
    const int64_t *b_off;    /* [nel+1] element offsets into out_b when p == 0 */
    int32_t *status;         /* [2] or NULL: atomically adds #elements where detJ > 0 fails
                                at some point (NaN included) and #elements with a non-finite
                                input or output */
    void *workspace;         /* mixed degree only: fem_workspace_bytes(nel) bytes, 256-B aligned */
    size_t workspace_bytes;
    const double *jac;       /* NULL, or supplied Jacobian terms (the NOJAC variant of section 4):
                                10 doubles per element and Gauss point, detJ then J^{-1} row-major
                                (J[a][b] = dx_a/dxi_b), point q = q1 + n q2 + n^2 q3; element e's
                                Nq = Ns records start at record e Nq (uniform p) or b_off[e]
                                (mixed degree, which then needs b_off even without out_b). They
                                replace the computation from geom, which then serves FIELD mode's
                                x_q only and may be NULL in the other modes. fem_jacobian_terms
                                writes them; any other source is taken as given. */
} fem_coeffs;

/* The set-up part of the host manager of section 4.2: make `device` current, query its
 * properties (compute units, shared-memory limits; section 4.2 sizes the launch from them),
 * build the FP64 reference tables for p = 1..7 (the arrays xi^Q, w^Q and phi^Q of section 2:
 * quadrature, 1-D Lagrange values and derivatives, the B^T operand tables in every precision)
 * and upload them once, so that later calls transfer no tables (section 4.2 keeps the shape
 * function table in global memory). Idempotent for the same device; FEM_EINVAL for a second
 * device. Not thread-safe; call before any other function. */
int fem_init(int device);

/* The tear-down part of the host manager of section 4.2: synchronise the device and release
 * the tables and staging buffers fem_init and fem_integrate_staged allocated. Afterwards every
 * call but fem_init returns FEM_ENOTINIT. */
int fem_finalize(void);

/* Integrate nel elements (Algorithm 2 of section 2 for each element, all elements in parallel:
 * elements over workgroups and entries of A^e over threads, section 4).
 *   nel    >= 0; nel == 0 returns FEM_OK and enqueues nothing
 *   p      1..7 for a uniform degree; 0 selects the per-element degrees coeffs->degree, which
 *          then also needs coeffs->a_off, coeffs->b_off (if out_b) and coeffs->workspace
 *   geom   [nel][8][3] FP64 vertex coordinates; may be NULL when coeffs->jac is given and the
 *          mode is not FEM_COEF_FIELD
 *   out_A  uniform p: [nel][Ns][Ns] row-major, unpadded; mixed: element e at a_off[e]
 *   out_b  uniform p: [nel][Ns]; mixed: element e at b_off[e]; may be NULL
 * Outputs are double for FEM_FP64 and float otherwise. */
int fem_integrate(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs, void *out_A,
                  void *out_b, void *stream);

/* Prismatic elements: the reference element of section 2 of the paper (Tables 1 and 2), the
 * prism T x [-1,1], T = {xi1, xi2 >= 0, xi1 + xi2 <= 1}, with shape functions i = t + Nt c
 * (Nt = (p+1)(p+2)/2, Ns = Nt (p+1): 6, 18, 40, 75, 126, 196, 288 for p = 1..7 as in Table 1):
 * the Lagrange basis of the complete degree-p polynomials on the triangle's principal lattice
 * (node t = (a/p, b/p), a + b <= p, b outer, a inner) times the 1-D Lagrange polynomial of GLL
 * node c in zeta. Quadrature (Table 1's N_Q = 6, 18, 48, 80, 150, 231, 336): the fully symmetric
 * degree-2p triangle rule with N_Q / (p+1) points times the (p+1)-point Gauss-Legendre rule in
 * zeta. The geometry is linear in the triangle and in zeta: vertex v = t + 3h of geom[e][6][3]
 * sits at triangle vertex t = (0,0), (1,0), (0,1) and zeta = -1 (h = 0) or +1 (h = 1).
 * Algorithm 2 of section 2 per element, eq. (sum_int) of section 5.1, as fem_integrate:
 *   nel >= 0, p = 1..7 (uniform), geom [nel][6][3] FP64, coeffs as for fem_integrate in the modes
 *   ELEMENT, FIELD and ELASTIC (coeffs->degree, a_off, b_off, workspace are ignored; coeffs->jac
 *   must be NULL: FEM_EINVAL otherwise), out_A [nel][Ns][Ns] (ELASTIC [nel][3][3][Ns][Ns]),
 *   out_b [nel][Ns] (ELASTIC [nel][3][Ns]) or NULL.
 * Asynchronous on `stream`; allocates nothing. */
int fem_integrate_prism(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs,
                        void *out_A, void *out_b, void *stream);

/* HOST copies of the prism's reference data (section 2, Tables 1-2): tri[ntq][3] = (xi1, xi2,
 * weight) of the triangle rule (ntq = N_Q / (p+1); weights sum to 1/2) and B[Nq][4][Ns] =
 * (phi_i, d phi_i/d xi1, d phi_i/d xi2, d phi_i/d zeta) at point q = qt + ntq qz. Either pointer
 * may be NULL. Needs no fem_init and no GPU. FEM_EDEGREE for p outside 1..7. */
int fem_prism_reference_tables(int p, double *tri, double *B);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): fem_integrate with the same arguments, layouts and
 * results, except that a mixed-degree call (p == 0) ignores coeffs->workspace and
 * coeffs->workspace_bytes and uses a static device array of the library instead (one per device,
 * about 16 MiB, held until the process ends, its address taken by fem_init). It allocates
 * nothing, by any route. Limit: a mixed-degree call takes at most FEM_NOALLOC_MAX_NEL elements,
 * more return FEM_ETOOBIG with nothing enqueued (uniform-degree calls need no scratch and take
 * any nel). The array keeps the last call's contents; every call clears what it needs zeroed by
 * a kernel of its own. All calls on one device share the one array, so mixed-degree calls that
 * overlap on one device (concurrent streams, host threads) race; serialise them. */
#define FEM_NOALLOC_MAX_NEL (1LL << 22)
int fem_integrate_noalloc(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs,
                          void *out_A, void *out_b, void *stream);

/* Jacobian terms for the NOJAC variant (section 4: the determinant and the 9 entries of the
 * inverse Jacobian of every element at every quadrature point, read by the integration instead
 * of recomputed): writes jac in the layout of fem_coeffs.jac, in FP64, from the trilinear map
 * of geom [nel][8][3]. p = 1..7 for a uniform degree (jac: [nel][Ns][10]); p = 0 takes
 * degree [nel] and the b_off scan of fem_mixed_offsets (jac: [b_off[nel]][10]; points of an
 * element whose degree is outside 1..7 are not written). Values equal those the integration
 * computes itself from the same vertices. Asynchronous on `stream`; allocates nothing. */
int fem_jacobian_terms(int64_t nel, int p, const double *geom, const int8_t *degree,
                       const int64_t *b_off, double *jac, void *stream);

/* Host-resident meshes (the end-to-end view of section 5.4, whose Tables 6 and 7 time the
 * transfer of inputs, the kernel and the transfer of results separately): integrates nel elements of uniform degree
 * p whose data live in HOST memory, in chunks of `chunk` elements over `nstreams` streams
 * (1..FEM_STAGED_MAX_STREAMS). Chunk c goes to stream c mod nstreams as {copy geometry and
 * records to the device, fem_integrate, copy A and b back}; with more than one stream the
 * copies of one chunk overlap the kernels of others. Host memory from hipHostMalloc (or
 * torch's pin_memory) lets the copy engines run asynchronously; pageable memory works but
 * serialises the copies.
 *   geom, coeffs->elem, coeffs->field, out_A, out_b  HOST pointers, layouts as for
 *          fem_integrate (uniform p, any coefficient mode); out_b may be NULL
 *   coeffs->status  HOST int32[2] or NULL: the counts over all chunks are added to it
 *   coeffs->degree, a_off, b_off and jac must be NULL (FEM_EINVAL otherwise)
 *   stats  HOST, may be NULL: wall time of the call and per-stage sums of event times
 * Blocks until the results are in out_A / out_b. The device staging buffers and streams are
 * allocated on the first call, grown when a larger chunk needs it, reused by later calls and
 * released by fem_finalize; concurrent calls are serialised. */
#define FEM_STAGED_MAX_STREAMS 8
typedef struct fem_staged_stats {
    double total_ms;     /* host wall time from the first enqueue to the last completion */
    double h2d_ms;       /* sums over chunks of the event times of each stage */
    double kernel_ms;
    double d2h_ms;
    int64_t h2d_bytes;   /* bytes moved each way */
    int64_t d2h_bytes;
    int64_t chunks;
} fem_staged_stats;
int fem_integrate_staged(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs,
                         void *out_A, void *out_b, int64_t chunk, int nstreams,
                         fem_staged_stats *stats);

/* Bytes of device workspace that a mixed-degree fem_integrate over nel elements needs: the
 * element ids classified by degree (section 4.2: the host manager splits the elements into
 * sets of equal degree) and the partial sums of fem_mixed_offsets. 0 for nel < 0. */
size_t fem_workspace_bytes(int64_t nel);

/* Output placement for a mesh of mixed degree (section 4.2: elements classified by degree; the
 * unpadded element matrices of section 4.1 then lie back to back): exclusive scans
 * a_off[e] = sum_{e' < e} Ns(e')^2 and b_off[e] = sum_{e' < e} Ns(e') over a
 * device degree array, nel + 1 entries each, computed on the device. `workspace` as for
 * fem_integrate. Degrees outside 1..7 count as 0 entries; fem_integrate skips such elements. */
int fem_mixed_offsets(int64_t nel, const int8_t *degree, int64_t *a_off, int64_t *b_off,
                      void *workspace, size_t workspace_bytes, void *stream);

/* One time step of the coefficient fields, on the device: with t = *step, if 0 <= t < nsteps,
 * theta_sm += deltas[t][s][m] for the 7 x 5 modes of `field` (reduced to [0, 2 pi)), then
 * *step = t + 1; otherwise nothing changes. deltas: [nsteps][7][5] FP64 phase increments
 * supplied by the caller (seeded, drawn on the host); field: the 175-double descriptor of
 * FEM_COEF_FIELD; step: one int32. All DEVICE pointers. Enqueues one small kernel and neither
 * allocates nor synchronises, so a stream capture of {fem_field_advance, fem_integrate}
 * replays as a time-step loop (time-dependent coefficients c^Q of section 2). */
int fem_field_advance(double *field, const double *deltas, int32_t nsteps, int32_t *step,
                      void *stream);

/* Gather a sample of the element matrices and load vectors into compact buffers, on the device
 * (section 5.4, Tables 6-7: results travel back to the host after integration; in a replayed
 * time step only a sample of them needs to). sel: [nrows][nsel] element ids; the row used is
 * (*step - 1) mod nrows, the step counter that fem_field_advance moved on earlier in the same
 * replay, or row 0 when step is NULL. a_off, b_off: the nel + 1 offsets of the source matrices
 * and vectors (fem_mixed_offsets; element e's matrix is A[a_off[e] .. a_off[e + 1])). A, b: the
 * outputs of fem_integrate in `precision`'s output type (FP64 for FEM_FP64, FP32 otherwise; b
 * may be NULL, then out_b must be NULL too). out_A, out_b: the selected elements' matrices and
 * vectors back to back in selection order, at most cap_A and cap_b entries written; ids outside
 * [0, nel) are skipped and take no space. All pointers except the scalars are DEVICE pointers.
 * Enqueues one kernel (nsel workgroups); allocates and synchronises nothing, so it can be
 * captured with {fem_field_advance, fem_integrate}. FEM_EINVAL on bad arguments. */
int fem_gather_sample(int64_t nsel, const int32_t *sel, int32_t nrows, const int32_t *step,
                      int64_t nel, const int64_t *a_off, const int64_t *b_off, const void *A,
                      const void *b, int precision, void *out_A, int64_t cap_A, void *out_b,
                      int64_t cap_b, void *stream);

/* HOST copies of the degree-p reference data the kernels use (section 2: quadrature points and
 * weights, and the 1-D factors of the shape functions): gauss_x[n], gauss_w[n] (the
 * (p+1)-point Gauss-Legendre rule), lobatto_x[n] (the nodes of the shape functions),
 * L[q][a] = l_a(gauss_x[q]) and D[q][a] = l_a'(gauss_x[q]), n = p+1. Any pointer may be NULL.
 * Needs no fem_init and no GPU. Returns FEM_EDEGREE for p outside 1..7. */
int fem_reference_tables(int p, double *gauss_x, double *gauss_w, double *lobatto_x, double *L,
                         double *D);

/* Kernel variants. Each (p, precision) is compiled in up to FEM_MAX_VARIANTS tile
 * configurations (elements per workgroup, waves per element, chunk depth of the contraction,
 * whether the column operand C = D_q B is produced cooperatively in LDS or per wave in
 * registers, whether the B^T table stays resident in LDS). Which one is fastest depends on p,
 * the precision and the device; section 4 motivates choosing the work assignment per degree.
 * fem_integrate launches the variant chosen for its (p, precision): a default measured on
 * MI355X until one of the calls below chooses another. The choice is process-wide and not
 * thread-safe.
 * p = 1 has one more variant, FEM_TRILINEAR_VARIANT(precision): not a tile configuration but
 * a vector-ALU kernel (8 x 8 x 32 per element is too small for the matrix cores; the element's
 * memory traffic bounds it): eight lanes per element, FP64 Jacobian terms and point matrices,
 * the sums in the precision's output type (FP64 for FEM_FP64, FP32 otherwise, which is at
 * least as accurate as the 16-bit products). It takes ELEMENT coefficients only and is the
 * default there; FIELD and ELASTIC calls use the tile variants.
 * p = 0 addresses the mixed-degree path (fem_integrate with p == 0), which has two variants:
 * 0 integrates every degree in one persistent launch (the work items of all degrees form one
 * index space, heaviest degree first; 256-thread workgroups throughout, each degree with the
 * tile chosen for it under key FEM_MIXED(p)); 1 (the default) issues one launch per degree, each
 * with the variant chosen for that degree.
 * FEM_MIXED(p), p = 1..7, addresses the tile degree p runs with inside that single launch: one
 * or two alternatives (variant 0 the default), each one of the 256-thread tile variants of the
 * degree's own launches (fem_mixed_variant names it). */
#define FEM_MAX_VARIANTS 7
#define FEM_TRILINEAR_VARIANT(precision) ((precision) == FEM_FP64 ? 1 : 5)

/* Variant keys of the prism of degree p (p = 1..7) in the calls below. */
#define FEM_PRISM(p) (10 + (p))

/* Variant keys of the tile of degree p (p = 1..7) inside the single mixed-degree launch. */
#define FEM_MIXED(p) (20 + (p))

/* Number of variants compiled for (p, precision), p = 0..7, FEM_PRISM(1..7) or FEM_MIXED(1..7) (>= 1),
 * FEM_EDEGREE or FEM_EINVAL (the work-assignment parameters of section 4.2 as compiled
 * alternatives). */
int fem_variant_count(int p, int precision);

/* The variant fem_integrate (fem_integrate_prism for p = FEM_PRISM(1..7)) launches for
 * (p, precision, mode) (section 4.2: parameters chosen per degree), or FEM_EDEGREE / FEM_EINVAL.
 * mode is a fem_coef_mode: the coefficient mode changes the per-point prologue, so each mode has
 * its own choice. */
int fem_get_variant(int p, int precision, int mode);

/* Choose the variant for (p, precision, mode) (section 4.2); FEM_ECONFIG if variant >=
 * fem_variant_count, or if it is the p = 1 vector-ALU variant and mode is not ELEMENT. Every
 * variant computes the same result to the precision's tolerance. */
int fem_set_variant(int p, int precision, int mode, int variant);

/* The tile configuration, as a variant number of degree p's own launches, that the single-launch
 * mixed-degree kernel currently runs degree p = 1..7 with for (precision, mode) (section 4.2:
 * per-degree parameters inside the one launch over all degree classes; the alternative chosen
 * under key FEM_MIXED(p)). FEM_EDEGREE / FEM_EINVAL on bad arguments. */
int fem_mixed_variant(int p, int precision, int mode);

/* Blocks of the elastostatics element matrix (section 5.1: 3 x 3 blocks of Ns x Ns) that an
 * ELASTIC call for degree p (1..7, or FEM_PRISM(1..7)) and precision integrates on the matrix
 * cores: 9, or 6 where the blocks below the diagonal are written as transposed copies of those
 * above (the major symmetry of c_ijkl). FEM_EDEGREE / FEM_EINVAL on bad arguments. Host only. */
int fem_elastic_blocks(int p, int precision);

/* Choose the work assignment of (p, precision, mode) by measurement (section 4.2 derives the
 * launch parameters per degree from the device's limits; here the compiled variants are timed
 * instead): time every variant on a seeded synthetic batch of nel elements in coefficient mode
 * `mode` (mildly distorted cubes; ELEMENT: CDR records, FIELD: rotations, loads and a seeded
 * field descriptor, ELASTIC: E, nu and body forces; for p = 0 degrees 1..7 drawn with weights
 * 8 - p, the timed call including the device bucketing, after the tile of every degree inside
 * the single launch has been tuned the same way (key FEM_MIXED(d) on a batch of about
 * nel (8 - d) / 28 elements of degree d, recorded in the same file); for p = FEM_MIXED(d) a
 * batch of degree d alone through the single mixed-degree launch; for p = FEM_PRISM(1..7)
 * mildly distorted prisms through fem_integrate_prism; ELASTIC needs p = 1..7 or a prism
 * key; 1 warm-up and 5
 * timed calls each, on a stream of its own), choose the fastest for (p, precision, mode), and,
 * if json_path is not NULL, record the choice and the times in that HOST file, keyed by
 * (architecture, p, precision, mode) (other entries of an existing file are kept). chosen
 * (HOST, may be NULL) receives the variant, times_ms (HOST [FEM_MAX_VARIANTS], may be NULL)
 * the mean milliseconds per call of each variant (-1 for a variant that does not take the
 * mode). Allocates and frees device memory for the
 * batch and synchronises; not for use under stream capture. */
int fem_autotune(int p, int precision, int mode, int64_t nel, const char *json_path, int *chosen,
                 double *times_ms);

/* Apply the choices recorded in a file written by fem_autotune (section 4.2: per-degree launch
 * parameters). FEM_ECONFIG if the file was written on another GPU architecture; entries naming
 * a variant that does not exist are skipped. applied (HOST, may be NULL) receives the number of
 * choices applied. */
int fem_load_tuning(const char *json_path, int *applied);

/* Static text for a status code of the argument and device checks of the host manager
 * (section 4.2). Never NULL. */
const char *fem_strerror(int status);

/* FEM_ABI_VERSION of the loaded library: the layout of fem_coeffs and of these calls (the
 * operation, Algorithm 2 of section 2 in the arrangement of section 4, is the same in every
 * version). */
int fem_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
