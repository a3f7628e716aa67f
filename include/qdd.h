/* qdd.h -- C ABI of the MI355X (gfx950) clover-Wilson Dirac operator and its
 * locally deflated, Schwarz-preconditioned flexible GCR solver.
 *
 * What it computes (arXiv:1011.0911, "Comparison of the mass preconditioned HMC
 * and the DD-HMC algorithm for two-flavour QCD"):
 *   - D = D_W + c_sw sum_{mu,nu} (i/4) sigma_{mu nu} F_{mu nu} + m     (Eq. 1),
 *     with m = 1/(2 kappa) - 4, D_W the nearest-neighbour Wilson operator
 *     -1/2 sum_mu [(1-g_mu) U_mu(x) d_{x+mu,y} + (1+g_mu) U_mu(x-mu)^dag d_{x-mu,y}] + 4;
 *   - its even-odd Schur complement Dhat = D_ee - D_eo D_oo^{-1} D_oe (Eq. 2;
 *     the paper's Q_S = D_ee^{-1} Dhat);
 *   - solves D psi = eta with the locally deflated Schwarz-preconditioned GCR
 *     the paper uses for its F2 inversions (Sect. 3 and 4, Table 1).
 *
 * Conventions: lattice L[0] x L[1] x L[2] x L[3], direction 0 = time; canonical
 * site index lex = ((x0*L1 + x1)*L2 + x2)*L3 + x3; parity (x0+x1+x2+x3) mod 2;
 * chiral Euclidean gamma basis g0 = [[0,-1],[-1,0]], gk = [[0,-i sk],[i sk,0]],
 * g5 = diag(1,1,-1,-1); the fermion boundary sign bc_time multiplies the hops
 * across the time boundary.
 *
 * Canonical arrays at the boundary are device pointers to complex128
 * (interleaved re, im doubles):
 *   links      U[lex][mu][a][b]                      (V*4*9 complex)
 *   spinors    psi[rhs][lex][spin][colour]           (nrhs*V*12 complex)
 *   even field psi_e[rhs][lex>>1][spin][colour]      (even sites only, nrhs*V/2*12)
 * Internal ("packed") fields, used by the hot-path calls qdd_dw_hat / qdd_dw,
 * are opaque device buffers of qdd_field_bytes() bytes made by qdd_pack_field.
 *
 * Ownership: the caller allocates every device buffer, including the workspace
 * of qdd_workspace_bytes() bytes handed to qdd_create; the library keeps
 * non-owning pointers into it and never allocates device memory itself.
 * Streams: every call is asynchronous on the stream given to qdd_create, except
 * where a host result is returned (set_params reads one flag, the solvers read
 * residual norms each iteration).  One context per host thread.
 * Errors: every call returns a qdd_status; qdd_last_error() describes the last
 * failure.  No call aborts or exits.  Arguments are validated before any HIP
 * call, so invalid geometry or sizes fail without touching the GPU.
 */
#ifndef QDD_H
#define QDD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QDD_OK = 0,
  QDD_EINVAL = -1,    /* invalid argument or geometry */
  QDD_ESTATE = -2,    /* call out of order (e.g. apply before set_params) */
  QDD_ESINGULAR = -3, /* a 6x6 clover block is not positive definite */
  QDD_ENOCONV = -4,   /* solver hit nmx iterations or a non-finite residual */
  QDD_EHIP = -5,      /* HIP runtime error */
  QDD_ENOWS = -6      /* workspace too small */
} qdd_status;

typedef enum { QDD_F64 = 0, QDD_F32 = 1, QDD_F16 = 2 } qdd_prec; /* F16 = FP16 storage, FP32 arithmetic */

typedef enum {
  QDD_PRECOND_NONE = 0, /* plain flexible GCR */
  QDD_PRECOND_SAP = 1,  /* Schwarz alternating procedure */
  QDD_PRECOND_DFL = 2   /* deflation + SAP (two-level) */
} qdd_precond;

typedef struct {
  int L[4];    /* L[0] = time extent; all even */
  int bc_time; /* -1 antiperiodic (default), +1 periodic */
} qdd_geom;

typedef struct {
  int max_nrhs;        /* largest right-hand-side batch of any call */
  /* Schwarz preconditioner */
  int sap_bs[4];       /* block extents; an even number of blocks per direction */
  int ncy;             /* SAP cycles per preconditioner call */
  int nmr;             /* minimal-residual steps per block solve */
  qdd_prec sap_prec;   /* arithmetic of the SAP sweeps (F64, F32, F16 storage) */
  /* local deflation */
  int dfl_Ns;          /* deflation vectors (0 = off) */
  int dfl_bs[4];       /* deflation block extents */
  int dfl_nit;         /* SAP inverse-iteration rounds in the subspace build */
  double dfl_coarse_tol; /* relative tolerance of the little-operator solve */
  int dfl_coarse_nmx;  /* iteration cap of the little-operator solve */
  /* outer flexible GCR (FP64) */
  int nkv;             /* Krylov vectors before a restart (<= 32) */
  int nmx;             /* iteration cap */
  double tol;          /* relative residual |eta - D psi| / |eta| */
  qdd_precond precond;
  int use_net;         /* 1: gauge-covariant network stage inside the preconditioner */
  int net_nl;          /* network layers */
  int net_ch[8];       /* channels ch[0] .. ch[nl] (ch[0] = ch[nl] = 1) */
  int net_terms;       /* BF16 terms per activation in the network's products when it is
                          applied (qdd_net_forward, the solver's network stage): 3 keeps
                          FP32 accuracy; 2 or 1 round each transported activation to 16
                          or 8 significant bits (relative error <= 2^-16, 2^-8), fewer
                          matrix-core operations; training always uses 3 */
  /* chronological inversion (Sect. 3): the solver keeps the last chrono_nv
     solutions of every right-hand-side slot and starts each qdd_solve from their
     least-squares combination (0 = off; at most 16 and at most nkv * max_nrhs) */
  int chrono_nv;
  /* deflation-subspace refresh: when a deflated qdd_solve needs more than
     dfl_refresh_iters outer iterations (0 = never) the subspace is refreshed
     after it, with dfl_refresh_nit rounds of SAP inverse iteration started from
     the current basis (as qdd_dfl_refresh) */
  int dfl_refresh_iters;
  int dfl_refresh_nit;
  /* 1: the workspace also holds the buffers of qdd_force (4 FP64 fields, the
     per-plane clover insertions and 2 even fields: 1392 bytes per site) */
  int force;
  /* Dirichlet block solver (qdd_block_solve): block extents (even, dividing the
     lattice); all 0 = no block solver.  Reserves the block-major links and clover
     blocks and eight FP64 vectors per rhs (about 2.1 KB per site per rhs) */
  int blk_bs[4];
} qdd_config;

typedef struct {
  int iters;        /* outer FGCR iterations */
  int restarts;
  int converged;    /* 1 if true relative residual <= tol */
  int fallbacks;    /* network stage rejected (plain SAP used instead) */
  double true_res;  /* |eta - D psi| / |eta| with FP64 D, at exit */
  double t_ms[8];   /* host-side stage times: 0 total, 1 preconditioner, 2 operator,
                       3 Gram-Schmidt, 4 coarse correction, 5 network, 6 SAP, 7 residual
                       restarts; kernels run asynchronously, so a stage's GPU time is
                       counted where the host next waits (the Gram-Schmidt reductions);
                       only index 0 is a GPU-inclusive wall time */
  double gpu_ms[4]; /* GPU time of the stages, from HIP events on the solver's stream:
                       0 preconditioner, 1 operator (with the FP32 -> FP64 conversion),
                       2 Gram-Schmidt and residual update, 3 the restarts (solution
                       update and true residual); shared by the rhs of a batch */
} qdd_solve_info;

typedef struct {
  int nblk;          /* blocks times right-hand sides solved */
  int converged;     /* how many reached |r| <= tol |b| */
  int breakdowns;    /* how many stopped on a zero BiCGstab denominator */
  int iters_max;     /* largest iteration count */
  double res_max;    /* largest final |r| / |b| */
  double t_ms;       /* GPU time of the solve (HIP events) */
} qdd_block_info;

typedef struct qdd_ctx qdd_ctx;

/* Fills *cfg with the defaults: max_nrhs 1, SAP 4^4 blocks, ncy 5, nmr 4, F32;
 * no deflation (Ns 0, blocks 4^4, nit 5, coarse tol 1e-6, nmx 2000);
 * nkv 16, nmx 2048, tol 1e-10, precond NONE; no network (3 layers 1-12-12-1,
 * 3 terms); no chronological inversion; no automatic refresh (2 rounds when
 * enabled). */
void qdd_config_default(qdd_config* cfg);

/* Workspace bytes needed for geometry + configuration; 0 if they are invalid. */
size_t qdd_workspace_bytes(const qdd_geom* geom, const qdd_config* cfg);

/* Creates a context on the current HIP device.  dev_ws: caller-owned device
 * buffer of ws_bytes (>= qdd_workspace_bytes), 256-byte aligned.  stream: a
 * hipStream_t (NULL = default stream). */
qdd_status qdd_create(const qdd_geom* geom, const qdd_config* cfg, void* dev_ws, size_t ws_bytes, void* stream,
                      qdd_ctx** out);
void qdd_destroy(qdd_ctx* ctx);
const char* qdd_last_error(const qdd_ctx* ctx);

/* Gauge ingest (canonical complex128 links, device pointer; the gauge field
 * U_mu(x) of Eq. 1): builds the parity-split hopping copies in FP64, FP32 and
 * FP16 with the boundary sign folded in.  Invalidates clover and deflation data. */
qdd_status qdd_set_gauge(qdd_ctx* ctx, const double* dev_links);

/* Clover setup (Eq. 1): F_{mu nu} from the clover leaves, A = (4+m) + c_sw
 * sum (i/4) sigma F as two Hermitian 6x6 blocks per site, their FP64 Cholesky
 * inverses, and FP32 / FP16 copies.  Synchronises to read the singularity flag:
 * QDD_ESINGULAR if any block is not positive definite. */
qdd_status qdd_set_params(qdd_ctx* ctx, double kappa, double csw);

/* Bytes of a packed field of `nrhs` right-hand sides (even_only: even sites). */
size_t qdd_field_bytes(const qdd_ctx* ctx, qdd_prec prec, int nrhs, int even_only);
/* canonical complex128 (device) -> packed field of precision prec (FP16 with a
 * per-site scale), and back. */
qdd_status qdd_pack_field(qdd_ctx* ctx, qdd_prec prec, int nrhs, int even_only, const double* canon, void* field);
qdd_status qdd_unpack_field(qdd_ctx* ctx, qdd_prec prec, int nrhs, int even_only, const void* field, double* canon);

/* out_e = Dhat in_e on packed even fields (Eq. 2), nrhs right-hand sides in one
 * pair of launches; the links and clover blocks are read once per site for all
 * of them. */
qdd_status qdd_dw_hat(qdd_ctx* ctx, qdd_prec prec, int nrhs, const void* in_e, void* out_e);
/* out = D in on packed full fields (Eq. 1). */
qdd_status qdd_dw(qdd_ctx* ctx, qdd_prec prec, int nrhs, const void* in, void* out);
/* Full D at one mass per right-hand side in one launch (Eq. 1): out_r = D(kappas[r]) in_r,
 * using that only the diagonal of the clover term, 1/(2 kappa), depends on kappa, so
 * D(kappa_r) = D(kappa) + (1/(2 kappa_r) - 1/(2 kappa)) with kappa that of qdd_set_params.
 * kappas: host array of nrhs positive values (nrhs <= 64); fields as for qdd_dw.
 * QDD_EINVAL for bad arguments, QDD_ESTATE before qdd_set_params. */
qdd_status qdd_dw_masses(qdd_ctx* ctx, qdd_prec prec, int nrhs, const double* kappas, const void* in, void* out);

/* psi = M_sap eta: ncy cycles of the two-colour Schwarz procedure with nmr
 * minimal-residual steps on the even-odd block operator of every block, in the
 * configured SAP precision (the Schwarz preconditioner of the solver the paper
 * uses for its inversions, Sect. 3).  Canonical complex128 full fields. */
qdd_status qdd_sap(qdd_ctx* ctx, int nrhs, const double* eta, double* psi);

/* Local deflation subspace of the solver's deflation (Sect. 3; its cost is
 * counted in the solve times of Sect. 4, Table 1): init holds dfl_Ns canonical
 * full fields (the random start vectors, supplied by the caller); dfl_nit rounds
 * of SAP inverse iteration, block orthonormalisation (FP64) and the little Dirac
 * operator (self + 8 face couplings per block, FP64). */
qdd_status qdd_dfl_build(qdd_ctx* ctx, const double* init);

/* Inspection of the deflation data of Sect. 3 (device pointers, either may be NULL): the
 * block-orthonormal basis as dfl_Ns canonical full fields, and the little Dirac
 * operator A[b][f][k][l] = <w_bk, D w_b'l> (complex128, nblk x 9 x Ns x Ns;
 * f = 0 the block with itself, f = 1 + 2 mu + dir the coupling through the
 * block's upper (dir 0) or lower (dir 1) face in direction mu; blocks numbered
 * lexicographically like sites).  Synchronises. */
qdd_status qdd_dfl_export(qdd_ctx* ctx, double* basis, double* little);
/* Solves the little system A c = f of the deflation (Sect. 3; device
 * [rhs][nblk][Ns] complex128) with the FP64 GCR of the preconditioner to
 * relative residual tol; *iters (host) gets the iteration count. */
qdd_status qdd_dfl_coarse_solve(qdd_ctx* ctx, int nrhs, const double* f, double* c, double tol, int* iters);
/* Reuses the deflation subspace of `src` (same gauge field, lattice, blocks, Ns)
 * at the mass of `dst` (several masses share one subspace, Sect. 4 and the
 * mass-preconditioned solves of Sect. 2): the basis is copied and the little operator shifted,
 * A_dst = A_src + (1/(2 kappa_dst) - 1/(2 kappa_src)) 1 on every block's self
 * coupling (exact for a block-orthonormal basis).  Synchronises. */
qdd_status qdd_dfl_share(qdd_ctx* dst, const qdd_ctx* src);

/* One application of the two-level preconditioner of the deflated solver (Sect. 3),
 * out = C r + M_sap(r - D C r) with C = W A^{-1} W^dag (canonical full fields). */
qdd_status qdd_dfl_precond(qdd_ctx* ctx, int nrhs, const double* r, double* out);

/* Solves D psi = eta (canonical full fields, nrhs right-hand sides, psi
 * overwritten) with FP64 flexible GCR and the configured preconditioner (the
 * locally deflated Schwarz-preconditioned GCR of Sect. 3-4 with precond DFL).
 * With chrono_nv > 0 the solve starts from the chronological guess and stores
 * its solutions; with dfl_refresh_iters > 0 a deflated solve that took more outer
 * iterations refreshes the subspace afterwards.  info: nrhs entries (host
 * memory) or NULL.  QDD_ENOCONV if any rhs fails. */
qdd_status qdd_solve(qdd_ctx* ctx, int nrhs, const double* eta, double* psi, qdd_solve_info* info);
/* As qdd_solve, but psi holds an initial guess on entry (warm start, as the
 * chronological inversion of Sect. 3 uses: the first residual is eta - D psi; a
 * guess that already meets tol returns at once with 0 iterations). */
qdd_status qdd_solve_guess(qdd_ctx* ctx, int nrhs, const double* eta, double* psi, qdd_solve_info* info);
/* The chronological guess (Sect. 3) for eta from the stored solutions (what qdd_solve
 * would start from), written to psi without solving; QDD_EINVAL with
 * chrono_nv = 0.  psi = 0 for a rhs slot with no stored solution. */
qdd_status qdd_chrono_guess(qdd_ctx* ctx, int nrhs, const double* eta, double* psi);
/* Forgets the solutions stored for the chronological inversion (chrono_nv > 0;
 * Sect. 3): the next qdd_solve starts from 0. */
qdd_status qdd_chrono_reset(qdd_ctx* ctx);
/* Refreshes the deflation subspace for the current operator (after qdd_set_gauge
 * or qdd_set_params changed it): dfl_refresh_nit rounds of SAP inverse iteration
 * started from the current basis, normalised after each round, then the block
 * orthonormalisation and the little operator as in qdd_dfl_build (Sect. 4,
 * Fig. 1: the subspace is updated along the trajectory).  QDD_ESTATE without a
 * basis built or shared before. */
qdd_status qdd_dfl_refresh(qdd_ctx* ctx);
/* Numbers of subspace builds and refreshes (automatic ones included) of ctx. */
qdd_status qdd_dfl_stats(const qdd_ctx* ctx, int* builds, int* refreshes);
/* Solves nsys independent systems (lattices, masses and batch sizes may all
 * differ) concurrently, each as qdd_solve does (the solver of Sect. 3-4; several
 * masses share one deflation subspace through qdd_dfl_share): each context (with
 * its own stream) runs its solve on a host thread of its own, so the work of all
 * systems is in flight at once and each stops at its own convergence.  eta[s], psi[s]: canonical fields of
 * system s; info[s]: nrhs[s] entries or NULL.  Returns the first failure. */
qdd_status qdd_solve_multi(qdd_ctx* const* ctxs, int nsys, const int* nrhs, const double* const* eta,
                           double* const* psi, qdd_solve_info* const* info);
/* The same systems solved by one outer flexible GCR loop (Sect. 3) in which
 * every stage is ONE launch over the workgroups of all systems still iterating:
 * the Schwarz face and half-sweep kernels, the full D, the precision
 * conversions and each Gram-Schmidt reduction and update.  A table in the
 * kernel arguments maps each workgroup to (system, its own workgroup number);
 * systems advance in lockstep through a restart cycle, a system whose
 * right-hand sides have all converged leaves the tables until the cycle ends,
 * and per-rhs device masks freeze converged right-hand sides.  Each system gets
 * exactly the result its own qdd_solve gives (same kernels, same reduction
 * blocking).  All work runs on the stream of ctxs[0].  Needs 1 to 12 contexts on
 * one device, all with the Schwarz preconditioner in one storage precision,
 * FP32 or FP16 (equal block volume and kernel variant), or all with none,
 * chrono_nv = 0; QDD_EINVAL with
 * the reason in ctxs[0]'s error text otherwise.  eta[s], psi[s], info[s] as for
 * qdd_solve_multi; QDD_ENOCONV if any rhs fails (its context holds the text). */
qdd_status qdd_solve_group(qdd_ctx* const* ctxs, int nsys, const int* nrhs, const double* const* eta,
                           double* const* psi, qdd_solve_info* const* info);
/* Solves Dhat psi_e = eta_e (Eq. 2; canonical even fields) with unpreconditioned
 * FP64 FGCR (the plain method). */
qdd_status qdd_solve_dhat(qdd_ctx* ctx, int nrhs, const double* eta_e, double* psi_e, qdd_solve_info* info);

/* ---- mass preconditioning (Sect. 2, Eqs. 2-5) ----
 * With Q = gamma5 D, Eq. 2 factorises det Q = det Q_ee det Q_oo det Q_S,
 * Q_S = 1 - Q_ee^{-1} Q_eo Q_oo^{-1} Q_oe, and Eq. 3 introduces
 * W(dm) = Q_S + dm; the effective action of Eq. 4 carries
 * -2 (log det Q_ee + log det Q_oo). */
/* *logdet_even, *logdet_odd (host) = log det Q_ee and log det Q_oo of the
 * current operator (qdd_set_params): the sums over the even and over the odd
 * sites of log det A(x) (det gamma5 = 1 on a site's 12 components), from the
 * Cholesky factors of the FP64 clover blocks, summed in a fixed order
 * (deterministic).  Synchronises.  QDD_ESTATE before qdd_set_params,
 * QDD_ESINGULAR if a block is not positive definite. */
qdd_status qdd_clover_logdet(qdd_ctx* ctx, double* logdet_even, double* logdet_odd);
/* out_e = W(dm) in_e = Q_S in_e + dm in_e (Eq. 3) on packed FP64 even fields
 * (qdd_pack_field, prec F64, even_only 1), nrhs right-hand sides.  Since the
 * gamma5 factors cancel, Q_S = A_e^{-1} Dhat: the FP64 Dhat apply, then the
 * even-site inverse clover blocks and the shift.  in_e and out_e must not
 * overlap (QDD_EINVAL otherwise); QDD_ESTATE before qdd_set_params. */
qdd_status qdd_apply_w(qdd_ctx* ctx, int nrhs, double dm, const void* in_e, void* out_e);
/* out_e = Q_S^{-1} phi_e by Eq. 5, Q_S^{-1} = P_e Q^{-1} Q_ee P_e: the configured
 * solver (as qdd_solve: FP64 flexible GCR, with deflation and SAP when
 * configured) solves D psi = (A_e phi_e on the even sites, 0 on the odd ones)
 * and out_e is the even half of psi.  The residual reported and tested is that
 * of Q_S itself, |phi_e - Q_S out_e| / |phi_e| (FP64 Dhat, inverse even clover
 * blocks); where it is above tol the same solve is run on it and the correction
 * added (at most twice); info.iters counts all of them.  phi_e, out_e:
 * canonical complex128 even fields (device), nrhs of them.  QDD_ENOCONV if a
 * residual stays above tol; other errors as for qdd_solve. */
qdd_status qdd_solve_qs(qdd_ctx* ctx, int nrhs, const double* phi_e, double* out_e, qdd_solve_info* info);
/* out_e = W(dm)^{-1} phi_e (Eq. 3, W(dm) = Q_S + dm, dm >= 0).  Since
 * W = A_e^{-1} (Dhat + dm A_e) and Dhat + dm A_e is the even-odd Schur complement
 * of D' = D with the even sites' clover term scaled by 1 + dm, the configured
 * solver solves D' psi = (A_e phi_e (+) 0) (its preconditioner is the one built
 * for D) and out_e is the even half of psi; residual, refinement, arguments and
 * errors as for qdd_solve_qs, with W(dm) in place of Q_S. */
qdd_status qdd_solve_w(qdd_ctx* ctx, int nrhs, double dm, const double* phi_e, double* out_e, qdd_solve_info* info);
/* Effective action of Eq. 4 with two pseudofermion fields phi1, phi2 (canonical
 * complex128 even fields, device):
 *   S_eff = -2 (log det Q_ee + log det Q_oo) + |W^{-1}(dm) phi1|^2 + |(1 + dm Q_S^{-1}) phi2|^2
 * (the dm/Q_S of Eq. 4 read as dm Q_S^{-1}).  chi1 = W^{-1}(dm) phi1 and
 * chi2 = Q_S^{-1} phi2 are returned in the caller's buffers (even fields; they are
 * what the pseudofermion forces consume); the two solves run as one batch of two
 * right-hand sides, so the context needs max_nrhs >= 2.  *s_eff (host) gets the
 * total, parts (host, 3 doubles, optional) the log-det term and the two
 * pseudofermion terms, info (2 entries, optional) the solves as in qdd_solve_w.
 * QDD_EINVAL for dm < 0, max_nrhs < 2 or chi1 == chi2; else errors as for
 * qdd_clover_logdet and qdd_solve_w. */
qdd_status qdd_action(qdd_ctx* ctx, double dm, const double* phi1, const double* phi2, double* chi1, double* chi2,
                      double* s_eff, double* parts, qdd_solve_info* info);
/* Forces of the effective action of Eq. 4 (the molecular-dynamics forces of
 * Sect. 2): the derivative of S_eff (as qdd_action, same phi1, phi2, dm) with
 * respect to every link, U_mu(x) -> exp(eps T^a) U_mu(x), along the eight
 * generators T^a = i lambda^a / 2 (Gell-Mann lambda^a).  terms selects the parts
 * of S_eff: bit 0 the log-det term (the clover-term force), bit 1 the phi1 term,
 * bit 2 the phi2 term (nothing for dm = 0).  The pseudofermion terms take two
 * batched solves of two right-hand sides with the configured solver: psi =
 * W(dm)^{-1} phi1 and xi = Q_S^{-1} phi2, then X = (Dhat + s A_e)^{-dag} w for
 * (s, w) = (dm, psi) and (0, phi2 + dm xi) through gamma5-hermiticity
 * (X = gamma5 W(s)^{-1} A_e^{-1} gamma5 w); the hopping and clover parts of the
 * derivative follow from these fields and their odd-site images.  force (device,
 * FP64): [V][4][8] in lexicographic site order, f^a of U_mu(x) at
 * (lex * 4 + mu) * 8 + a, overwritten.  info: 4 entries (psi, xi, X_1, X_2) or
 * NULL.  QDD_EINVAL for dm < 0, terms outside 1..7, a context created without
 * config.force or with max_nrhs < 2; QDD_ESTATE before qdd_set_params; solver
 * errors as for qdd_solve_w. */
qdd_status qdd_force(qdd_ctx* ctx, double dm, const double* phi1, const double* phi2, int terms, double* force,
                     qdd_solve_info* info);
/* Dirichlet block solves (the block inversions of the DD-HMC forces, which the
 * paper does with BiCGstab, Sect. 3): D_Lambda psi = eta on every block Lambda of
 * extent config.blk_bs, D_Lambda being D restricted to the block (hops that leave
 * the block dropped).  Each block's source is reduced to its even sites
 * (b = eta_e - D_eo,L A_o^{-1} eta_o), BiCGstab on the block's even-odd Schur
 * complement runs from zero until |r| <= tol |b| or maxit iterations, and the odd
 * sites are reconstructed; FP64.  One workgroup solves one (block, rhs) in a
 * single launch.  eta, psi: nrhs canonical complex128 full fields (device).
 * blk_iters / blk_res (host, nrhs * nblk entries, rhs-major, blocks in
 * lexicographic block order, or NULL): iterations (-1 after a breakdown) and final
 * |r|/|b| per block.  QDD_EINVAL for a context without blk_bs, nrhs outside
 * 1..max_nrhs, tol <= 0 or maxit < 1; QDD_ESTATE before qdd_set_params; QDD_ENOCONV
 * if a block did not converge (psi holds the last iterate, info the counts). */
qdd_status qdd_block_solve(qdd_ctx* ctx, int nrhs, const double* eta, double* psi, double tol, int maxit,
                           int* blk_iters, double* blk_res, qdd_block_info* info);

/* ---- learned preconditioner stage (configuration use_net = 1; an extension
 * the paper does not have, placed inside its deflated solver of Sect. 3) ----
 * A gauge-covariant parallel-transport convolution network N with net_nl
 * layers and channels net_ch[0..nl]; layer: out_c(x) = sum_{c',d} W[d][c][c']
 * (T_d in_{c'})(x), d = 0 identity, d = 1+2mu forward transport U_mu(x)
 * psi(x+mu), d = 2+2mu backward transport U_mu(x-mu)^dag psi(x-mu), W a complex
 * 4x4 spin matrix.  Weights: complex FP32 (device, interleaved), layer after
 * layer, each W[d][c][c'][s][s'] row-major; they are used in BF16, activations
 * in FP32.  Inside the deflated preconditioner:
 * v = C r + N(r1) + M_sap(r2), r1 = r - D C r, r2 = r1 - D N(r1); for every
 * right-hand side whose |r2| > |r1| (or not finite) N is dropped (counted in
 * qdd_solve_info.fallbacks), so the plain method is always the floor. */
qdd_status qdd_net_num_weights(const qdd_ctx* ctx, int64_t* n);
qdd_status qdd_net_set_weights(qdd_ctx* ctx, const float* w);
qdd_status qdd_net_get_weights(qdd_ctx* ctx, float* w);
/* Sets net_terms (1, 2 or 3; see qdd_config) for the later network
 * applications of this context; QDD_EINVAL otherwise. */
qdd_status qdd_net_set_terms(qdd_ctx* ctx, int terms);
/* The solver's network stage runs in the first `calls` preconditioner
 * applications of every solve (each outer FGCR iteration applies the
 * preconditioner once to the whole batch) and is skipped after them, so that
 * later iterations cost what the method without the network costs; 0 (the
 * default) = every application.  QDD_EINVAL for calls < 0. */
qdd_status qdd_net_set_calls(qdd_ctx* ctx, int calls);
/* out = N(in), canonical complex128 full fields (one field). */
qdd_status qdd_net_forward(qdd_ctx* ctx, const double* in, double* out);
/* Loss l = sum_i |N(r_i/|r_i|) - e_i/|r_i||^2 / sum_i |e_i/|r_i||^2 over nb pairs
 * (canonical complex128, device, at most 8) and, if grad != NULL, its complex
 * gradient dl/dRe W + i dl/dIm W (device, FP32 complex, qdd_net_num_weights). */
qdd_status qdd_net_loss_grad(qdd_ctx* ctx, int nb, const double* r, const double* e, double* loss, float* grad);
/* One Adam step (lr; beta 0.9, 0.999) on a mini-batch of nb pairs given as
 * packed FP32 full fields (as written by qdd_solve_harvest). */
qdd_status qdd_net_train_step(qdd_ctx* ctx, int nb, const void* r, const void* e, float lr, double* loss);
/* Solves nrhs right-hand sides like qdd_solve, but with the plain method (no
 * network stage even where one is configured), and records, at every outer
 * iteration and for every right-hand side still iterating, r_k and
 * e_k = psi* - psi_k as packed FP32 full fields (qdd_field_bytes(ctx, QDD_F32,
 * 1, 0) bytes each, consecutive) into the caller's buffers, up to max_pairs;
 * *npairs gets the count and pair_rhs (host, max_pairs ints, optional) the
 * right-hand side of each pair.  The iteration that converges is not recorded.
 * e_pairs must hold max_pairs FP64 fields (qdd_field_bytes(ctx, QDD_F64, 1, 0)
 * each): the iterates stay in FP64 until psi* is known; the FP32 errors are
 * returned packed at its front. */
qdd_status qdd_solve_harvest(qdd_ctx* ctx, int nrhs, const double* eta, double* psi, qdd_solve_info* info,
                             void* r_pairs, void* e_pairs, int max_pairs, int* npairs, int* pair_rhs);

/* ---- launch tuning and measurement (extensions: the autotuner and the roofline
 * measurement of the GPU kernels; no passage of the paper) ----
 * Launch shape of a kernel family (kernel: 0 = Dhat, 1 = D, 2 = the Schwarz
 * half-sweep; prec: qdd_prec).  For kernel 2 only nr is used, the kernel variant
 * of FP32 / FP16 storage (block, xcd and sb must be 0): 1 one lane per site with
 * its links and clover block in registers, the right-hand sides one after
 * another; 2 one workgroup per (block, right-hand side), a lane per even/odd
 * site pair; 3 one workgroup per block and group of 4 right-hand sides with
 * the block's links (FP16: and clover blocks) staged in LDS; 4 (FP16 only)
 * one workgroup per block and pair of right-hand sides with the block's links
 * staged in LDS (two workgroups per CU).  FP64 has a
 * single kernel (qdd_get_launch reports nr 0).  The default is 3 for FP16 and 1
 * for FP32.  For kernels 0 and 1:
 * block threads (64..256, multiple of 64); nr right-hand sides per lane (1, 2,
 * 4; the links are loaded once for all of them), or nr = 0 (Dhat only): the
 * staged variant, where a workgroup reads the links and clover of its tile of
 * sb sites into LDS once and its block/sb lanes per site loop over all
 * right-hand sides (tile LDS: 108 complex per site, at most 64 KiB); xcd: block
 * walk (0 linear; 1 every XCD takes a contiguous slab of the lattice; 2 slabs
 * whose tiles are walked time slice first, so time and x1 neighbours stay in
 * the XCD's L2; 3 slabs of L1/8 x1 planes through all time slices, walked
 * one time slice after the other); for Dhat with nr = 1 plus 4: streaming
 * (non-temporal) loads of the links and clover blocks, plus 8: streaming load
 * of the site's own spinor and store of the output: data a pass touches once,
 * kept from evicting the neighbour spinors from the L2; plus 16: compressed
 * links, of which only the first two rows are read (12 of 18 reals) and the
 * third is rebuilt as the conjugate cross product (an SU(3) identity; the time
 * boundary sign of the stored link is put back); for Dhat with nr = 2 or 4
 * in FP32 (nr 2) or FP16 (nr 2, 4), plus 32: rhs-vector loads, a lane reads
 * the nr right-hand sides of a spinor component (and their FP16 scales) as one
 * word of at most 16 bytes, with the streaming and compression bits (4, 8, 16)
 * as for nr = 1; it applies to interleaved batches whose size is a multiple of
 * nr, other operands take the plain kernels; for Dhat with nr >= 1, plus 64:
 * pass B walks its tiles backwards (every XCD's range from its end), so it
 * starts with the odd-site intermediate pass A wrote last; sb sites per block
 * (0 = block): the block/sb lane groups of a
 * block take further right-hand sides of the same sites.  QDD_EINVAL for shapes
 * outside these ranges. */
qdd_status qdd_set_launch(qdd_ctx* ctx, int kernel, qdd_prec prec, int block, int nr, int xcd, int sb);
qdd_status qdd_get_launch(const qdd_ctx* ctx, int kernel, qdd_prec prec, int* block, int* nr, int* xcd, int* sb);

/* Autotuner: times every candidate launch shape of `kernel` (0 = Dhat on packed
 * even fields, 1 = D on packed full fields) for this precision and batch size
 * on the given packed fields (`reps` timed repetitions each, HIP events on the
 * context stream), installs the fastest in the context and returns its mean
 * duration in *best_ms.  Kernel 2 times each Schwarz half-sweep variant on whole
 * preconditioner calls M_sap in (in: packed FP64 full fields, out: packed FP32
 * full fields of nrhs right-hand sides; prec must be the configured FP32 or FP16
 * SAP precision).  `out` is overwritten; synchronises. */
qdd_status qdd_autotune(qdd_ctx* ctx, int kernel, qdd_prec prec, int nrhs, const void* in, void* out, int reps,
                        float* best_ms);

/* qdd_dw_hat, repeated `reps` times with HIP events recorded on the context's
 * stream before pass A, between the passes and after pass B; returns the mean
 * duration of each pass in milliseconds (synchronises). */
qdd_status qdd_dw_hat_timed(qdd_ctx* ctx, qdd_prec prec, int nrhs, const void* in_e, void* out_e, int reps,
                            float* ms_pass_a, float* ms_pass_b);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same apply as
 * qdd_dw_hat (same kernels, bit-identical result), but the odd-site
 * intermediate of the two passes lives in a static device array of the library
 * (64 MiB per GPU, held from the first call on a GPU until the process ends)
 * instead of the context's workspace.  It needs nrhs * V/2 * 12 complex
 * elements of the precision (plus one FP32 scale per site and rhs for F16,
 * after a 256-byte aligned offset); QDD_EINVAL if that exceeds 64 MiB, or if
 * the current device is not the context's.  Calls no allocating routine.
 * Every call on one GPU shares the array: calls that overlap on one GPU (on
 * different streams, or from several host threads) race; calls ordered on one
 * stream do not.  Nothing needs clearing between calls (pass A writes all of
 * the intermediate before pass B reads it). */
qdd_status qdd_dw_hat_static(qdd_ctx* ctx, qdd_prec prec, int nrhs, const void* in_e, void* out_e);

/* Plain device-to-device copy of `bytes` (multiple of 16) with 16-byte vector
 * loads and stores on `stream`: the HBM bandwidth reference of the benchmarks. */
qdd_status qdd_copy(void* dst, const void* src, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif
