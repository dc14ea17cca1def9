/*
 * qdw.h -- C ABI of libqdw: the O(a)-improved Wilson-clover Dirac operator and its
 * solvers on one AMD Instinct MI355X (gfx950).
 *
 * In the paper's introduction, applying the Dirac operator to a spinor field -- a
 * bandwidth-bound relative of a sparse matrix-vector product -- is a key kernel of
 * lattice field theory, and the paper analyses the two solvers that spend their time
 * in it: the mixed-precision conjugate gradient on the normal
 * equations (Sec. 2, cgne) and the Schwarz-alternating-procedure preconditioned flexible
 * GCR (Sec. 3, fgcr with the settings of Table 2). This library provides exactly that
 * path as hand-written HIP kernels.
 *
 * Operator (standard Wilson-Sheikholeslami-Wohlert form):
 *   (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ s U_mu(x) (1 - g_mu) psi(x+mu)
 *                                         + s U_mu(x-mu)^+ (1 + g_mu) psi(x-mu) ]
 *   A(x) = (4 + m0) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x)
 * with U = exp(i theta) V, V in SU(3), theta the U(1) angle (QCD+QED, charge 1), s = bc_t
 * on hops across the time boundary, chiral gamma basis with gamma_5 = diag(1,1,-1,-1).
 *
 * Conventions for every entry point:
 *  - Pointers marked (device) are device memory of the current HIP device; (host) are
 *    host memory. The caller owns every buffer it passes; the library never frees or
 *    retains them beyond the call (except where stated).
 *  - `stream` is a hipStream_t (NULL = default stream). All device work of a call is
 *    enqueued on it. Calls that return solver information synchronise the stream.
 *  - Return value: QDW_OK (0) on success, a negative QDW_E* code otherwise; the
 *    message of the last failure on the calling thread is qdw_last_error(). No C++
 *    exception crosses this boundary.
 *  - A qdw_op may be used from one stream at a time (its reduction scratch is shared).
 *
 * Field layout ("eo-SoA", what dw_apply and the solvers read and write): sites split by
 * parity (x0+x1+x2+x3) mod 2, even first (the paper's even-odd ordering, Fig. 3 left).
 * Within a parity the site with lexicographic index lex = ((x0*L1 + x1)*L2 + x2)*L3 + x3
 * sits at position i = lex/2; positions are grouped in blocks of 64 (the count per parity
 * padded to a multiple of 64), and a block stores 16-byte chunk 0 of its 64 sites, then
 * chunk 1, ...: [parity][i/64][chunk][i%64]. A site's 24 reals (12 complex, index
 * spin*3 + colour, interleaved re/im) fill 12 chunks in FP64, 6 in FP32, 3 in FP16/BF16.
 * qdw_field_bytes gives a field's size; qdw_pack / qdw_unpack convert from and to the
 * canonical layout [V][4][3] complex128. The padding positions hold no site.
 */
#ifndef QDW_H
#define QDW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* storage precision of a spinor field; arithmetic is FP64 for QDW_F64, FP32 otherwise */
typedef enum {
    QDW_F64 = 0,   /* binary64 storage and arithmetic                          */
    QDW_F32 = 1,   /* binary32 storage and arithmetic                          */
    QDW_F16S = 2,  /* binary16 storage, binary32 arithmetic                    */
    QDW_BF16S = 3  /* bfloat16 storage, binary32 arithmetic                    */
} qdw_prec;

enum {
    QDW_OK = 0,
    QDW_EINVAL = -1,       /* invalid argument (null pointer, bad size or enum)       */
    QDW_EDEVICE = -2,      /* a HIP call failed                                        */
    QDW_ENOTUNITARY = -3,  /* a link is not in SU(3) to 1e-10 (qdw_create)             */
    QDW_EBLOCK = -4,       /* SAP block size does not tile the lattice as required     */
    QDW_ENOMEM = -5,       /* device allocation failed                                 */
    QDW_EWORKSPACE = -6    /* workspace too small                                      */
};

typedef struct {
    int T, L1, L2, L3; /* extents; all must be even, direction 0 is time            */
    int bc_t;          /* -1 antiperiodic or +1 periodic in time; space is periodic  */
} qdw_lattice;

typedef struct qdw_op qdw_op; /* opaque: compressed links and clover, all precisions */

/* Message of the last error on this thread ("" if none). */
const char* qdw_last_error(void);

/* Device and host bytes an operator on lattice `lat` keeps: qdw_op_device_bytes(lat) for
 * the compressed links, the clover blocks (their inverses, and the compact form the D
 * kernels read) in all four precisions and the reduction scratch, about 4.1 kB per site
 * (8.6 GB at 32^3 x 64); 0 for an invalid lattice.
 * qdw_op_host_bytes() for the scalars the host reads back (8 kB). */
size_t qdw_op_device_bytes(const qdw_lattice* lat);
size_t qdw_op_host_bytes(void);

/* Build an operator on the current device in memory the caller provides.
 *  su3   (device) complex128 [V][4][3][3], canonical site order: SU(3) part of U_mu(x)
 *  theta (device) float64 [V][4]: U(1) angle of U_mu(x)
 *  m0, csw: bare mass and Sheikholeslami-Wohlert coefficient.
 *  dev_mem (device) at least qdw_op_device_bytes(lat) bytes, any alignment;
 *  host_mem (host) at least qdw_op_host_bytes() bytes, pinned (hipHostMalloc or a pinned
 *  torch tensor) so that the solvers' scalar read-backs overlap with device work.
 * Both blocks stay owned by the caller, must outlive the operator, and are used by it
 * alone; the library allocates no memory of its own (the opaque qdw_op handle is a small
 * host struct). Checks that every su3 matrix is unitary with unit determinant to 1e-10
 * (QDW_ENOTUNITARY otherwise), then stores the two-row compressed links and builds the
 * clover blocks A_+-(x) in FP64 (Sec. 1 names O(a)-improved Wilson fermions); FP32,
 * FP16 and BF16 copies are derived by rounding to nearest even. QDW_EWORKSPACE when a
 * block is too small. The input buffers may be freed once this call has returned (it
 * synchronises `stream`). */
int qdw_create(const qdw_lattice* lat, const double* su3, const double* theta, double m0,
               double csw, void* dev_mem, size_t dev_bytes, void* host_mem, size_t host_bytes,
               void* stream, qdw_op** out);
/* Releases the handle (after a device synchronisation); the caller then frees its blocks. */
int qdw_destroy(qdw_op* op);

/* Number of lattice sites, and bytes of one eo-SoA spinor field in precision `prec`. */
long qdw_volume(const qdw_op* op);
size_t qdw_field_bytes(const qdw_op* op, qdw_prec prec);

/* Canonical complex128 [V][4][3] (device) <-> eo-SoA field in `prec` (device).
 * Down-conversion rounds to nearest even. */
int qdw_pack(const qdw_op* op, const double* canonical, void* eo, qdw_prec prec, void* stream);
int qdw_unpack(const qdw_op* op, const void* eo, double* canonical, qdw_prec prec, void* stream);

/* out = D in, and out = D^+ in = gamma_5 D gamma_5 in (the normal-equation solver of
 * Sec. 2 applies both per step). `in` and `out` are distinct eo-SoA fields (device) of
 * precision `prec`; the links and clover term are read in the same precision (FP16 and
 * BF16 storage: binary32 arithmetic). Deterministic: no atomics. */
int dw_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream);
int dw_dag_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream);

/* Uncompressed control for the link storage (Sec. 1: the hopping term reads every link;
 * not an operation of the paper): the FP64 operator with each link read as its full 3x3
 * matrix, 18 reals, instead of two rows and det U with the third row rebuilt in the kernel.
 * qdw_full_links_bytes: device bytes of the full FP64 links of op (0 for a null op).
 * qdw_set_full_links: forms them in dev_mem (device, caller-owned, 16-byte aligned, at
 * least qdw_full_links_bytes; op keeps using it until qdw_destroy or the next call) from
 * op's compressed FP64 links, the third row as d conj(row0 x row1) like the D kernels;
 * asynchronous on stream. dw_apply_full_links: out = D in (dagger != 0: D^+ in), FP64
 * eo-SoA fields (device, distinct), in a one-lane-per-site kernel with a plain hop loop on
 * the walk of op's FP64 shape (128-site tiles in chunks of 4 slices when that shape is the
 * marching form); QDW_EINVAL before qdw_set_full_links. Results equal dw_apply's to the
 * last bits of FP64 rounding. */
size_t qdw_full_links_bytes(const qdw_op* op);
int qdw_set_full_links(qdw_op* op, void* dev_mem, size_t bytes, void* stream);
int dw_apply_full_links(qdw_op* op, const void* in, void* out, int dagger, void* stream);

/* Even-odd reduced operator (the matrix of Sec. 3 is stored even sites first, Fig. 3
 * left; its Schur complement on the even sites): out_e = D^ in_e with
 * D^ = A_ee - D_eo A_oo^-1 D_oe, and D^+ = gamma_5 D^ gamma_5. Only the even half of `in`
 * is read; the even half of `out` receives the result and its odd half is overwritten
 * with A_oo^-1 D_oe in_e (scratch). The inverses of the odd-site clover blocks are formed
 * at qdw_create in FP64 (Gauss-Jordan with pivoting) and stored in every precision. */
int dw_schur_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream);
int dw_schur_dag_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream);

/* out[r] = D in[r] for r < nrhs (1 <= nrhs <= 64) in one launch: several right-hand sides
 * on one gauge field (Sec. 2 and 3 solve one system per source; the batch shares the
 * operator). in, out: host arrays of device eo-SoA fields of precision prec; no output may
 * alias any input. Workgroups of different right-hand sides on the same tile run side by
 * side, so the links and clover blocks of a tile come from HBM about once for the batch.
 * Results equal dw_apply on each field. */
int dw_apply_multi(qdw_op* op, const void* const* in, void* const* out, int nrhs,
                   qdw_prec prec, void* stream);

/* Device scratch (bytes) qdw_autotune needs: two fields of precision prec per right-hand
 * side. 0 on bad arguments. */
size_t qdw_autotune_workspace_bytes(const qdw_op* op, qdw_prec prec, int nrhs);
/* Autotuner of the D kernel for this operator (not from the paper): times every shape --
 * workgroup size (64 or 128 sites per parity), walk chunk (1, 2, 4, ..., 64 time slices,
 * dividing T), hop-loop form (plain or software-pipelined), tile order (walk 0: tiles of a
 * time slice in index order; 1: x1 slabs innermost, so the x1 neighbours of a tile are
 * loaded by nearby workgroups) and form (march 0: one workgroup per tile and slice; 1: a
 * workgroup marches through the chunk's slices of its tile and hands the time hops on
 * through LDS, so that they are read from memory once) -- for precision prec and nrhs
 * right-hand sides on the stream, keeps the fastest in op (used by dw_apply,
 * dw_apply_multi and the solvers from then on), and writes a one-line report (best shape,
 * then every candidate's time in ms as [ts,nt,pipe,walk,march]=ms) to report (host, may be
 * NULL). Times on two scratch fields per right-hand side filled with a fixed non-zero
 * pattern, in work (device, qdw_autotune_workspace_bytes bytes, clobbered); the two timing
 * events it creates are destroyed before it returns; synchronises the stream. Results do
 * not depend on
 * ts, nt or walk; the hop-loop forms and the marching form are separately compiled and
 * may differ in the last bit. */
int qdw_autotune(qdw_op* op, qdw_prec prec, int nrhs, void* work, size_t work_bytes,
                 char* report, size_t report_len, void* stream);
/* Shapes at qdw_create: FP64 and FP32 march on 64-site tiles with the longest walk chunk
 * (at most 32, dividing T) that still gives at least 512 workgroups (FP64 plain, FP32
 * pipelined hop loop); FP16 / BF16 storage: the plain one-lane-per-site form on 128-site
 * tiles, nt = 2.
 * Set / read the D kernel's shape for precision prec by hand (ts 64 or 128, nt in 1..64
 * dividing T, pipe 0 or 1, walk 0 or 1, march 0 or 1; shape5 = {ts, nt, pipe, walk,
 * march}); QDW_EINVAL for anything else. */
int qdw_set_dw_shape(qdw_op* op, qdw_prec prec, int ts, int nt, int pipe, int walk, int march);
int qdw_get_dw_shape(const qdw_op* op, qdw_prec prec, int* shape5);

/* Fused BLAS-1 on eo-SoA fields of one precision (device), every reduction accumulated in
 * binary64 (Sec. 2.1: reduction variables in binary64 whatever the working type) in a
 * fixed order, so results are bitwise reproducible. qdw_norm2 and qdw_cdot write their
 * result to host memory and synchronise the stream.
 *   qdw_axpby: y = a x + b y (real a, b)
 *   qdw_norm2: *out = |x|^2
 *   qdw_cdot:  out[0] + i out[1] = x^+ y */
int qdw_axpby(qdw_op* op, double a, const void* x, double b, void* y, qdw_prec prec,
              void* stream);
int qdw_norm2(qdw_op* op, const void* x, qdw_prec prec, double* out, void* stream);
int qdw_cdot(qdw_op* op, const void* x, const void* y, qdw_prec prec, double* out, void* stream);
/* y = s x between precisions (distinct fields; down-conversion rounds to nearest even) */
int qdw_convert(qdw_op* op, const void* x, qdw_prec px, void* y, qdw_prec py, double s,
                void* stream);

/* Result of a solve. */
typedef struct {
    int status;          /* >= 0: converged, number of regular steps (the paper's `status`,
                            Fig. 1); -1: nmx steps did not suffice; -2: stagnation (no
                            progress, Sec. 2: the residual stalls once the working type is
                            exhausted); -3: a non-finite value appeared                    */
    int nreset;          /* reset steps (CGNE) / restarts (GCR) performed                  */
    int n_dw_hi;         /* applications of D or D^+ in FP64                               */
    int n_dw_lo;         /* applications of D or D^+ in a lower precision (incl. SAP blocks
                            counted as one full-lattice application per colour sweep)     */
    int n_steps;         /* regular steps executed (equals status when converged)         */
    double rel_res_true; /* |eta - M psi| / |eta| recomputed in FP64 at exit, M = D^+D
                            (cgne_solve) or D (GCR solvers)                                */
    double t_sec;        /* wall time of the call, host clock                              */
} qdw_info;

/* Settings of the normal-equation solver (Sec. 2, openQ*D's cgne). */
typedef struct {
    double res;      /* target |eta - D^+ D psi| / |eta|                                   */
    int nmx;         /* maximal number of regular CG steps                                  */
    qdw_prec inner;  /* QDW_F64: plain FP64 CG. QDW_F32 / QDW_F16S / QDW_BF16S: regular
                        steps in that storage precision (binary32 arithmetic, binary64
                        reductions), reset steps in FP64                                    */
    double delta;    /* reset when the recursive residual fell by this factor since the last
                        reset. < 0: default, 10 eps of `inner` when keep_p = 0 (the paper's
                        reset, Fig. 1: about the working type's epsilon) and 0.1 when
                        keep_p = 1; 0: only when the target is reached or progress stalls  */
    int keep_p;      /* 1: a reset keeps the search direction (reliable update) as long as
                        the recursive residual stayed within 30 % of the true one, else
                        restarts; 0: every reset restarts CG from the new residual          */
    int cascade;     /* 1: precision cascade (Sec. 2.1: start in a 16-bit type until the
                        residual falls below a constant times its epsilon, continue in a
                        32-bit type until that is exhausted, finish in binary64): `inner` is
                        ignored; phases BF16 storage -> FP32 -> FP64, each a CG on the
                        current FP64 residual D^+ D delta = eta - D^+ D psi, psi += delta,
                        until |eta - D^+ D psi| / |eta| <= cascade_c eps(type) (Table 1
                        epsilons) or the phase stagnates; the FP64 phase finishes to res.
                        n_dw_hi then counts every FP64 application, n_dw_lo the BF16 and
                        FP32 ones; nreset counts resets and phase switches. 0: off           */
    double cascade_c;  /* the constant of the phase switch (default 1 when <= 0)           */
    int schur;       /* 1: solve the even-odd reduced normal equations D^+ D^ psi_e = eta_e
                        (D^ = A_ee - D_eo A_oo^-1 D_oe, see dw_schur_apply) instead of
                        D^+ D psi = eta: only the even halves of eta and psi are used, the
                        odd half of psi is set to zero, and rel_res_true refers to the
                        reduced system. Works with every inner precision and the cascade.
                        0: the full operator                                                */
} qdw_cgne_params;

/* Device workspace (bytes) cgne_solve needs for these settings. 0 on bad arguments. */
size_t qdw_cgne_workspace_bytes(const qdw_op* op, const qdw_cgne_params* prm);

/* Solve D^+ D psi = eta from psi = 0 (Sec. 2). eta and psi are distinct FP64 eo-SoA
 * fields (device); work is device memory of at least qdw_cgne_workspace_bytes bytes
 * (caller-owned scratch, clobbered). Regular steps keep their scalars in device memory;
 * the host reads |r|^2 one step late to decide on resets and termination. On return
 * psi holds the solution (also when status < 0: the best iterate), *info (host) the
 * outcome; the stream is synchronised. Non-convergence is reported in info->status,
 * not as an error code. */
int cgne_solve(qdw_op* op, const void* eta, void* psi, const qdw_cgne_params* prm, void* work,
               size_t work_bytes, qdw_info* info, void* stream);

/* Preconditioners of the flexible GCR solver. */
enum {
    QDW_PRECOND_NONE = 0,  /* identity: plain GCR, the paper's (ncy, nmr) = (0, 0)          */
    QDW_PRECOND_SAP = 1,   /* Schwarz alternating procedure (Sec. 3)                          */
    QDW_PRECOND_NN = 2,    /* learned gauge-covariant network (not from the paper)            */
    QDW_PRECOND_NN_SAP = 3, /* network while it reduces the GCR residual, then SAP            */
    QDW_PRECOND_SAP_ADAPTIVE = 4, /* adaptive SAP (Sec. 3.2): ncy and nmr are maxima; a cycle
                                    stops the application when it did not lower |rho|; a
                                    block's MR stops after >= 4 steps when |r_b| > sap_alpha
                                    times its previous value, when |r_b| grew, or when
                                    |r_b| < res |eta| / (number of blocks)                    */
    QDW_PRECOND_SAP_EO = 5 /* SAP whose block problems are solved on their even-odd reduced
                              form (as sap_eo_apply); nmr MR steps on the reduced block
                              operator per block solve                                     */
};

/* Settings of the SAP-preconditioned flexible GCR (Sec. 3.1, Table 2). The large and the
 * reduction data type (ldtype, rdtype) are binary64; sdtype is the small type of the
 * SAP block solves. */
typedef struct {
    double res;          /* desired relative residual |eta - D psi| / |eta|               */
    int nmx;             /* maximal number of GCR steps                                    */
    int nkv;             /* Krylov vectors generated before a restart (1..16)              */
    int ncy;             /* SAP cycles per preconditioner application                      */
    int nmr;             /* MR steps per block per cycle                                   */
    int bs[4];           /* block extents (T, L1, L2, L3 order). Each divides the lattice
                            extent with an even number (>= 2) of blocks per direction; the
                            block holds 64, 128, 192 or 256 sites (QDW_EBLOCK otherwise)     */
    qdw_prec sdtype;     /* QDW_F32, QDW_F16S or QDW_BF16S storage for the SAP fields      */
    int precond;         /* QDW_PRECOND_*                                                  */
    const void* nn_weights; /* (device) network weights for QDW_PRECOND_NN / _NN_SAP        */
    double sap_alpha;    /* QDW_PRECOND_SAP_ADAPTIVE: the MR exit factor alpha (0.9 in
                            Sec. 3.2); ignored otherwise                                    */
} qdw_sap_gcr_params;

/* Device workspace (bytes) sap_gcr_solve needs (2 nkv + 2 FP64 fields plus the
 * preconditioner's). 0 on bad arguments. */
size_t qdw_sap_gcr_workspace_bytes(const qdw_op* op, const qdw_sap_gcr_params* prm);

/* Solve D psi = eta from psi = 0 with flexible GCR restarted every nkv steps (Sec. 3.1).
 * eta, psi: distinct FP64 eo-SoA fields (device); work: device scratch of at least
 * qdw_sap_gcr_workspace_bytes. On return psi holds the solution and *info (host) the
 * outcome (status = GCR steps, nreset = restart steps, rel_res_true = |eta - D psi|/|eta|
 * of the final FP64 restart step); n_dw_lo counts SAP work as ncy*nmr block-operator
 * sweeps of the full lattice per preconditioner application. Synchronises the stream. */
int sap_gcr_solve(qdw_op* op, const void* eta, void* psi, const qdw_sap_gcr_params* prm,
                  void* work, size_t work_bytes, qdw_info* info, void* stream);

/* Several flexible-GCR solves at once (not from the paper: batching across right-hand
 * sides and lattices): problem j solves D_j psi_j = eta_j with operator ops[j] (ops may
 * repeat: the right-hand sides of one operator are solved together; operators may have
 * different lattice volumes), all with settings p (precond QDW_PRECOND_NONE,
 * QDW_PRECOND_SAP or QDW_PRECOND_SAP_EO). Each solve takes the same steps, with the same
 * arithmetic, as sap_gcr_solve on its own; all convergence decisions are made on the
 * device, and finished solves are gated off by flags the kernels read on entry.
 *
 * A batch plan captures `cycles` restart cycles (nkv steps and the restart step each) of
 * the whole batch once, as one HIP graph whose branches are the operators' groups, in
 * the caller's workspace `work` (device, qdw_sap_gcr_batched_workspace_bytes bytes; the
 * plan keeps using it until destroyed). The plan owns 1 + (number of operators) HIP
 * streams and as many events, used only to capture, and the graph; it allocates no
 * memory. A solve with the plan launches the graph on the caller's stream until every
 * solve has finished, reading the flags after each launch: one launch and one host wait
 * when `cycles` cycles suffice. etas, psis: host arrays of n device FP64 eo-SoA fields
 * (psi distinct from each other and from every eta); infos: n results (host; t_sec = wall
 * time of the solve call); launches (host, may be NULL): graph launches made. The same
 * plan serves any number of solves (one at a time). qdw_batch_capture_ms: time taken to
 * capture and instantiate the graph. */
typedef struct qdw_batch qdw_batch;
size_t qdw_sap_gcr_batched_workspace_bytes(qdw_op* const* ops, int n,
                                           const qdw_sap_gcr_params* p);
int qdw_batch_create(qdw_op* const* ops, int n, const qdw_sap_gcr_params* p, int cycles,
                     void* work, size_t work_bytes, qdw_batch** out);
int qdw_batch_solve(qdw_batch* b, const void* const* etas, void* const* psis, qdw_info* infos,
                    int* launches, void* stream);
double qdw_batch_capture_ms(const qdw_batch* b);
int qdw_batch_destroy(qdw_batch* b);
/* One-shot form: a plan of one cycle per launch, one solve, the plan destroyed; graph_ms
 * (host, may be NULL) receives its capture time. */
int sap_gcr_solve_batched(qdw_op* const* ops, const void* const* etas, void* const* psis, int n,
                          const qdw_sap_gcr_params* p, void* work, size_t work_bytes,
                          qdw_info* infos, double* graph_ms, void* stream);

/* ---- learned gauge-covariant preconditioner (not from the paper) ----------------------
 * Three linear parallel-transport layers, 1 -> 8 -> 8 -> 1 spinor channels:
 *   out_a(x) = sum_{p=0..8} sum_b W_p[a][b] (T_p in_b)(x),
 *   T_0 = 1, T_{+mu} v(x) = s U_mu(x) v(x+mu), T_{-mu} v(x) = s U_mu(x-mu)^+ v(x-mu),
 * path order p = 0, +t, -t, +x1, -x1, +x2, -x2, +x3, -x3; W_p[a][b] a complex 4x4 spin
 * matrix, so the network commutes with gauge transformations. Weights (device, FP32
 * complex, interleaved re/im): layer after layer, each [9][Cout][Cin][4][4] (spin row,
 * spin column), qdw_nn_weight_count() complex numbers in all. Channel mixing runs on the
 * matrix cores: bf16 operands with FP32 accumulation, or FP32 operands when
 * f32_mixing != 0 (for gradient checks). Gradients are real gradients:
 * dL/dRe z + i dL/dIm z. Used by sap_gcr_solve with QDW_PRECOND_NN / QDW_PRECOND_NN_SAP. */
int qdw_nn_weight_count(void);
/* device workspace of nn_forward (training = 0) or nn_backward (training = 1) */
size_t qdw_nn_workspace_bytes(const qdw_op* op, int training);
/* out = N(in); in, out FP64 eo-SoA fields (device) */
int nn_forward(qdw_op* op, const float* weights, const void* in, void* out, int f32_mixing,
               void* work, size_t work_bytes, void* stream);
/* For L with real gradient gout = dL/dRe N(in) + i dL/dIm N(in) (FP64 field): dW (device,
 * 2 * qdw_nn_weight_count() floats, overwritten) and gin = dL/dRe in + i dL/dIm in. */
int nn_backward(qdw_op* op, const float* weights, const void* in, const void* gout, float* dW,
                void* gin, int f32_mixing, void* work, size_t work_bytes, void* stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, step >= 1, lr) on the batch mean of the loss
 * over nbatch (residual rho_k, error err_k = D^-1 rho_k) pairs of eo-SoA fields of
 * precision pair_prec (QDW_F64, QDW_F32 or QDW_BF16S; host arrays of device pointers):
 *   loss_kind 0: |N(rho) - err|^2 / |err|^2            (error space)
 *   loss_kind 1: |D (N(rho) - err)|^2 / |D err|^2      (the same error in the D-norm, i.e.
 *                the residual |D N(rho) - rho| a GCR step would leave; gradient through
 *                D^+ D with the library's FP32 operator)
 * Weights updated in place; adam: 4 * qdw_nn_weight_count() floats of state (zero before
 * step 1); *loss (host) = the batch loss before the update. work: at least
 * qdw_nn_workspace_bytes(op, 1) + 8 * qdw_nn_weight_count() + 512 bytes. */
int nn_train_step(qdw_op* op, float* weights, float* adam, int step, double lr,
                  const void* const* rho, const void* const* err, int nbatch, qdw_prec pair_prec,
                  int loss_kind, double* loss, void* work, size_t work_bytes, void* stream);

/* Adaptive SAP (Sec. 3.2) as one preconditioner application phi = M rho: at most ncy_max
 * cycles, stopping after the first cycle that did not lower |r| (r = rho - D phi, the
 * residual the cycles maintain); every block's MR loop runs at most nmr_max steps and
 * stops after the step that (1) makes >= 4 steps and leaves |r_b| > alpha times its value
 * one step before, (2) increases |r_b|, or (3) brings |r_b| below tol (absolute, in the
 * units of rho); blocks with |r_b| < tol at the start take no step. *cycles (host, may be
 * NULL) receives the cycles run (synchronises the stream); mr_steps (device, may be NULL)
 * receives the MR steps of every block, int[ncy_max][2][number of blocks / 2] (colour-0
 * blocks, then colour-1 blocks, each in block-index order); entries of cycles not run are
 * left as they were. Workspace as for sap_apply. */
int sap_adaptive_apply(qdw_op* op, const void* rho, void* phi, int ncy_max, int nmr_max,
                       double alpha, double tol, const int bs[4], qdw_prec sdtype, void* work,
                       size_t work_bytes, int* cycles, int* mr_steps, void* stream);

/* Device workspace (bytes) of sap_apply for storage precision sdtype. */
size_t qdw_sap_workspace_bytes(const qdw_op* op, qdw_prec sdtype);

/* phi = M_SAP rho: ncy Schwarz cycles (Sec. 3, Fig. 2), each solving every colour-0
 * block then every colour-1 block by nmr minimal-residual steps on the block operator
 * (hops leaving the block dropped, Fig. 3), from phi = 0. rho, phi: distinct FP64
 * eo-SoA fields (device); internally stored in sdtype, scaled to unit component size.
 * ncy = 0 copies rho. Errors: QDW_EBLOCK for an unsupported block size. */
int sap_apply(qdw_op* op, const void* rho, void* phi, int ncy, int nmr, const int bs[4],
              qdw_prec sdtype, void* work, size_t work_bytes, void* stream);

/* sap_apply without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the SAP fields live in a static device array of qdw_sap_noalloc_max_bytes() bytes
 * (24 MiB) that each GPU the library runs on holds until the process ends; its device
 * address is looked up on the first call on each device. Same kernels and results as
 * sap_apply; no allocation of any kind. QDW_EWORKSPACE when the lattice needs more than
 * the maximum (qdw_sap_workspace_bytes > 24 MiB: above about 174,000 sites with FP16/BF16
 * storage, 87,000 with FP32). Every call on one GPU shares that GPU's array (its contents
 * are whatever the last call left; everything the application reads is written first):
 * calls that overlap on one GPU, from several streams or threads, race. Like sap_apply
 * it reads |rho| back to the host (synchronises the stream). */
size_t qdw_sap_noalloc_max_bytes(void);
int sap_apply_noalloc(qdw_op* op, const void* rho, void* phi, int ncy, int nmr, const int bs[4],
                      qdw_prec sdtype, void* stream);

/* As sap_apply, with every block problem D_b chi = r_b solved through its even-odd
 * reduction (the site-diagonal clover term A, the in-block hops between the parities):
 * r^_e = r_e - D_eo A_oo^-1 r_o; nmr MR steps from 0 on the reduced block operator
 * A_ee - D_eo A_oo^-1 D_oe give chi_e; chi_o = A_oo^-1 (r_o - D_oe chi_e), which leaves the
 * odd half of the block residual at zero. Parity is the site's parity on the whole lattice.
 * Same arguments, workspace and errors as sap_apply. */
int sap_eo_apply(qdw_op* op, const void* rho, void* phi, int ncy, int nmr, const int bs[4],
                 qdw_prec sdtype, void* work, size_t work_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* QDW_H */
