/*
 * sos.h -- optimized Schwarz subdomain solves for the gravity equation on one
 * MI355X (gfx950).
 *
 * Problem (Sec. 2): Delta(Phi) = -4 pi G drho on a box, discretised with 27-node
 * Q2 hexahedra on an nx*ny*nz grid of equal box elements, homogeneous Dirichlet
 * or Neumann data per outer face.
 * Method (Sec. 3): non-overlapping Schwarz iteration with Robin transmission
 * conditions of zeroth order (operator p), Jacobi order, one Robin datum per
 * directed interface face, exchanged after every outer iteration. Every outer
 * iteration solves all subdomain problems with diagonally preconditioned
 * conjugate gradients (Sec. 6), on the GPU.
 *
 * Conventions
 *   - Every function returns 0 (SOS_OK) or a negative error code; none throws
 *     or aborts. sos_last_error() describes the last failure of the calling
 *     thread.
 *   - Element arrays: length nx*ny*nz, index ex + nx*(ey + ny*ez).
 *   - Node arrays: length (2nx+1)(2ny+1)(2nz+1), index ix + Nx*(iy + Ny*iz),
 *     Nx = 2nx+1, Ny = 2ny+1 (element vertices plus edge, face and cell
 *     mid-points).
 *   - Subdomain s = px + Px*(py + Py*pz). Directed face (s <- j) carries the
 *     Robin datum s receives from neighbour j; faces are numbered by s, then
 *     axis (x, y, z), then side (lower, upper). See sos_faces().
 *   - Pointers inside the descriptor structs are HOST pointers. Pointer
 *     arguments of sos_solve/sos_solve_load/sos_apply_local/sos_get_state/
 *     sos_set_state are DEVICE pointers on the context's device, caller-owned,
 *     contiguous, FP64 unless stated. Work is enqueued on opts.stream.
 *   - The library allocates its workspaces in sos_setup and frees them in
 *     sos_destroy. A context is not thread-safe; one context per stream.
 */
#ifndef SOS_H
#define SOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sos_ctx sos_ctx; /* opaque, owned by the library */

enum {
  SOS_OK = 0,
  SOS_EINVAL = -1,      /* bad argument or unsupported geometry             */
  SOS_ENOMEM = -2,      /* device or host allocation failed                 */
  SOS_EHIP = -3,        /* a HIP runtime call failed                        */
  SOS_ENOCONV = -4,     /* max_outer reached; phi and stats still written   */
  SOS_EBREAKDOWN = -5,  /* an inner CG broke down: non-positive p'Ap, a
                           non-finite value (e.g. NaN in the load), or a
                           team member that gave up at the team barrier;
                           detected at the next convergence check, after
                           which the solve stops (stats are written, the
                           broken subdomain keeps its iterate)            */
  SOS_ESTATE = -6       /* call out of order (e.g. no GPU, context unusable)*/
};

enum { SOS_DIRICHLET = 0, SOS_NEUMANN = 1 };

/* Arithmetic of the inner subdomain solves. The Robin data, the subdomain
 * iterates, the local residuals and the global residual are always FP64. */
enum { SOS_FP64 = 0, SOS_FP32_INNER = 1 };

/* How the inner CG solves are launched.
 *   SOS_STEPWISE: the host drives every CG step; one launch per step covers
 *                 all subdomains (apply + p'q, then update + r'z, r'r).
 *   SOS_BATCHED:  one fused kernel per outer iteration runs every subdomain's
 *                 complete CG solve (each workgroup owns a subdomain and
 *                 stops on its own criterion), and the outer iterations
 *                 between two convergence checks are replayed as one HIP
 *                 graph when use_graph is set. */
enum { SOS_STEPWISE = 0, SOS_BATCHED = 1 };

typedef struct {
  int32_t ne[3];    /* elements per axis, >= 1                               */
  double len[3];    /* box lengths, > 0                                      */
  int32_t bc[6];    /* x-, x+, y-, y+, z-, z+ : SOS_DIRICHLET or SOS_NEUMANN  */
} sos_mesh;

typedef struct {
  int32_t nparts[3];      /* subdomains per axis, 1 <= nparts[d] <= ne[d]     */
  const int32_t* cuts[3]; /* nparts[d]-1 strictly increasing element indices
                             in (0, ne[d]); NULL = equal split (ne divisible) */
} sos_partition;

/* Transmission operator of every directed face (Sec. 3): order 0 is p
 * (weak form p M_F), order 2 is p + q d^2/dtau^2 read with the symbol p + q k^2
 * (weak form p M_F + q K_F, K_F the tangential stiffness of the face with a
 * natural condition at the face's edges). */
typedef struct {
  int32_t order;     /* 0 or 2                                                 */
  double p0;         /* p of every directed face if p == NULL, > 0            */
  double q0;         /* q of every directed face if q == NULL (order 2), >= 0 */
  const double* p;   /* optional: per directed face, sos_faces() order        */
  const double* q;   /* optional (order 2): per directed face                 */
} sos_robin;

typedef struct {
  int32_t precision;   /* SOS_FP64 or SOS_FP32_INNER                          */
  int32_t mode;        /* SOS_STEPWISE or SOS_BATCHED                         */
  int32_t max_outer;   /* outer iteration limit (default 100000)              */
  int32_t max_inner;   /* CG iteration limit per subdomain solve (default 500)*/
  int32_t check_every; /* outer iterations between global residual checks (1)*/
  int32_t use_graph;   /* SOS_BATCHED only: replay check_every iterations as a
                          HIP graph (default 1)                               */
  double inner_tol;    /* CG stop: ||r_k|| <= inner_tol * ||r_0||, r_0 the
                          local residual of the current outer iterate
                          (default 1e-2 for FP32_INNER, 0 for FP64)           */
  double inner_abs;    /* and/or ||r_k|| <= inner_abs * ||b_s||, b_s the local
                          right-hand side (default 1e-10 for FP64, 0 for FP32)*/
  double G;            /* gravitational constant (default 6.672e-11, Sec. 2)  */
  void* stream;        /* hipStream_t; NULL = default stream                  */
  int32_t block;       /* SOS_BATCHED workgroup size; 0 = autotune: the first
                          batched solve times the candidate block shapes of
                          the fused kernel and keeps the fastest, cached in
                          $SOS_TUNE_CACHE (default ~/.cache/sos_autotune.jsonl)
                          per subdomain geometry, precision and inner tolerance
                          (only when block and team are both 0: a search with
                          either fixed neither reads nor writes the cache)   */
  int32_t team;        /* SOS_BATCHED blocks per subdomain in the fused kernel
                          (1..8; each owns a z-range, one team barrier per CG
                          iteration); 0 = autotune (with block)              */
  int32_t timing;      /* 1: time every fused-kernel launch with HIP events
                          (launches eagerly: events inside a graph are not
                          readable)                                           */
  int32_t wave_rows;   /* with block != 0: 1 = each wave of the fused kernel
                          owns whole x-rows of the plane (one workgroup
                          barrier per plane; EINVAL if block/64 waves of
                          64 x cols columns cannot cover every subdomain's
                          plane that way); the autotuner tries both forms  */
  int32_t resident;    /* 1 (default): the FP32 fused kernel may keep the CG
                          direction p and the correction x (or x alone) in
                          LDS for the whole launch where they fit (uniform
                          z-ranges; with block != 0 it does, the autotuner
                          tries both); 0: never                             */
  int32_t march;       /* axis every subdomain is marched along (set up once):
                          0 (default) z, or for a subdomain whose x-y node
                          plane exceeds 4096 nodes the axis across its
                          smallest node plane; 1, 2, 3: x, y, z for all.
                          The other two axes keep their global order; see
                          sos_axes                                         */
  int32_t schedule;    /* 1 (default): with one block per subdomain, each
                          launch of the fused CG kernel takes the subdomains
                          in decreasing order of the work of their previous
                          inner solve ((iterations + 1) x nodes), so long
                          solves start first; 0: fixed order, largest
                          subdomain first                                  */
} sos_opts;

typedef struct {
  int32_t outer_iters;    /* outer iterations performed                         */
  int32_t checks;         /* global residual evaluations                        */
  int64_t inner_iters;    /* CG iterations summed over subdomain solves         */
  double rel_residual;    /* ||f - K u||_2 / ||f||_2 over unknowns at the end   */
  double seconds;         /* wall time of the solve                             */
  double kernel_ms;       /* timing = 1: summed duration of the fused CG kernel
                             (SOS_BATCHED) or of the CG step kernels (STEPWISE) */
  int64_t kernel_launches;/* number of launches summed in kernel_ms             */
  double kernel_bytes;    /* algorithmic bytes of those launches: SOS_BATCHED
                             12 words per CG iteration and local unknown (a
                             PCG iteration with its dot products fused into the
                             operator sweep) + per solve the read of x and the
                             FP64 update of u; SOS_STEPWISE the 10 vectors its
                             two kernels read and write per iteration          */
  int32_t block;          /* workgroup size used by the fused CG kernel         */
  int32_t cols_per_thread;/* x-y columns per thread of the fused CG kernel      */
  int32_t team;           /* blocks per subdomain of the fused CG kernel (the
                             largest team; see sos_teams)                      */
  int32_t wave_rows;      /* 1: each wave of the fused CG kernel owns whole
                             x-rows of the plane (one barrier per plane)       */
  int32_t resident;       /* the fused CG kernel keeps in LDS: 1 p and x,
                             2 x alone (p and x do not fit), 0 neither         */
} sos_stats;

/* Fill *opts with defaults for the given precision. */
int sos_opts_default(sos_opts* opts, int32_t precision);

/* Set up the Robin-Schwarz method of Sec. 3 on a box partition: validate
 * mesh/partition/Robin data (SOS_EINVAL: cuts not strictly increasing inside
 * (0, ne), a zero-width subdomain, p <= 0, q < 0, all outer faces Neumann,
 * bad options), build subdomain and directed-face descriptors (one Robin
 * datum per directed interface face), allocate device workspaces on the
 * current HIP device (SOS_ENOMEM), SOS_ESTATE without a usable device. Every
 * subdomain's node plane across its marched axis (opts.march) must hold at
 * most 4096 nodes (SOS_EINVAL otherwise). *out is NULL on
 * failure; on success the caller releases it with sos_destroy. */
int sos_setup(const sos_mesh* mesh, const sos_partition* part, const sos_robin* robin,
              const sos_opts* opts, sos_ctx** out);

/* Batch of `copies` independent copies of the same problem in one context
 * (1 <= copies <= 4096), for evaluating many transmission conditions at once
 * (the stochastic search of Sec. 4 scores candidate coefficients by the
 * convergence of the Schwarz iteration; Sec. 5 runs such evaluations on the
 * GPU). Copy c holds subdomains c*n_sub .. (c+1)*n_sub - 1 and directed faces
 * c*n_faces .. in the order of one copy; robin->p / robin->q, when given,
 * hold copies*n_faces values in that order (a different condition per copy).
 * Every kernel launch covers all copies. Vectors (local layout, lambda) and
 * phi_nodes (copies * nodes, copy-major) are concatenated copy after copy;
 * drho_elem is one field shared by every copy. The stopping quantity of a
 * solve is the largest relative residual over the copies. sos_solve_load and
 * sos_adjoint return SOS_EINVAL on such a context. sos_setup is
 * sos_setup_batch with copies = 1. */
int sos_setup_batch(const sos_mesh* mesh, const sos_partition* part, int32_t copies,
                    const sos_robin* robin, const sos_opts* opts, sos_ctx** out);

/* Relative residual ||f - K u~|| / ||f|| of every copy at the last global
 * residual evaluation (host memory, copies values). */
int sos_batch_residuals(sos_ctx* ctx, double* res);

/* Convergence rate of every copy: loads drho, starts from u = 0, lambda = 0,
 * runs n_first outer iterations, records each copy's relative residual r1,
 * runs to n_second and records r2; rates[c] = (r2/r1)^(1/(n_second-n_first))
 * (NaN if not finite). best = the copy of the smallest finite rate (ties: the
 * lower index). res_first / res_second / best / stats may be NULL; host
 * memory. SOS_EBREAKDOWN if no rate is finite. */
int sos_batch_rates(sos_ctx* ctx, const double* drho_elem, int32_t n_first, int32_t n_second,
                    double* rates, double* res_first, double* res_second, int32_t* best,
                    sos_stats* stats);

/* Replace the transmission coefficients of Sec. 3 (p, and q for order 2)
 * on every directed face, keeping the partition and the load (SOS_EINVAL as
 * in sos_setup; the context is unchanged on error). The outer state (u,
 * lambda) is kept; a following solve starts from zero anyway. */
int sos_set_robin(sos_ctx* ctx, const sos_robin* robin);

/* Replace the run options (precision is fixed at setup). */
int sos_set_opts(sos_ctx* ctx, const sos_opts* opts);

/* The directed interface faces (s <- j) of the partition, one Robin datum
 * each (the many-subdomain reading of Sec. 3's two-subdomain exchange).
 * *n receives their number; if s_j_axis != NULL it receives 4 int32 per face:
 * s, j, axis, side (host memory, caller-owned, 4*n entries). */
int sos_faces(const sos_ctx* ctx, int32_t* n, int32_t* s_j_axis_side);

/* Local axis order of every subdomain: perm[3*s + a] = the global axis (0 x,
 * 1 y, 2 z) of local axis a; local axis 2 is the one the kernels march along
 * (host memory, 3*n_sub entries). */
int sos_axes(const sos_ctx* ctx, int32_t* perm);

/* Team sizes of the batched fused CG kernel, one per subdomain (host memory,
 * n_sub entries, sos_layout order): the number of workgroups that share the
 * subdomain's inner solve (Sec. 6 solves each subdomain with one diagonally
 * preconditioned CG; a team splits its z-planes and meets at one barrier per
 * CG iteration). The autotuner picks them per size bucket: subdomains whose
 * node counts differ by more than 1.5x fall into three buckets of equal
 * width in log size, each with its own team size. */
int sos_teams(const sos_ctx* ctx, int32_t* teams);
/* Set them (1..8, at most the subdomain's z-planes; SOS_EINVAL otherwise):
 * the current block shape and these teams are used from now on without
 * autotuning, until sos_set_opts changes a launch option. */
int sos_set_teams(sos_ctx* ctx, const int32_t* teams);

/* Layout of the concatenated subdomain vectors: n_sub; if offsets != NULL it
 * receives n_sub+1 int64 offsets, if dims != NULL 3*n_sub int32 node counts
 * along each subdomain's local axes 0, 1, 2 (sos_axes: global x, y, z unless
 * a subdomain marches along another axis) and if lo != NULL 3*n_sub int32
 * global node indices (x, y, z) of each subdomain's first local node. Local
 * node (i, j, k) of s sits at offsets[s] + i + n0*(j + n1*k). Face f's datum
 * (sos_get_state) sits at face_off[f] if face_off != NULL (n_faces+1 int64),
 * its nodes along the face's tangential global axes, the lower one fastest. */
int sos_layout(const sos_ctx* ctx, int32_t* n_sub, int64_t* offsets, int32_t* dims,
               int32_t* lo, int64_t* face_off);

/* Solve the gravity equation of Sec. 2, Delta(Phi) = -4 pi G drho, with the
 * Robin-Schwarz iteration of Sec. 3 (subdomain solves by diagonally
 * preconditioned CG, Sec. 6) for a per-element density anomaly drho (kg/m^3,
 * device, n_elem FP64): f_s = 4 pi G sum over s's own elements of
 * drho_e int phi_i. Iterates until
 * the global relative residual ||f - K u~||/||f|| <= tol (checked every
 * check_every outer iterations; u~ the average of the subdomain copies) and
 * writes u~ to phi_nodes (0 on Dirichlet nodes). Starts from u = 0, lambda = 0.
 * Returns SOS_ENOCONV if max_outer is reached, or if the best residual has not
 * improved by 1% for 2000 outer iterations (stagnation, e.g. a tol below the
 * floor that an absolute inner tolerance leaves); phi and stats are still
 * written. */
int sos_solve(sos_ctx* ctx, const double* drho_elem, double tol, double* phi_nodes,
              sos_stats* stats);

/* sos_solve for a nodal load f (Sec. 2's weak right-hand side over all
 * nodes, device, FP64; values on Dirichlet nodes ignored), split among the
 * subdomain copies of every node in equal parts (the same fixed point as the
 * element-ownership split of sos_solve). Returns and errors as sos_solve;
 * SOS_EINVAL on a context of several copies. */
int sos_solve_load(sos_ctx* ctx, const double* f_nodes, double tol, double* phi_nodes,
                   sos_stats* stats);

/* Adjoint of sos_solve for a functional J(Phi) of the solution (Sec. 2: the
 * load is linear in drho, f = 4 pi G B drho with B_ie = int_e phi_i; K is
 * symmetric). Given dJ_dphi_nodes = dJ/dPhi over all nodes (device, FP64;
 * Dirichlet entries ignored), solves K psi = dJ/dPhi with the same Schwarz
 * iteration and options (tol relative to ||dJ/dPhi||) and writes
 *   dJ_ddrho_elem[e] = 4 pi G sum_i psi_i int_e phi_i      (device, FP64, n_elem)
 * and, if psi_nodes != NULL, psi over all nodes (device, 0 on Dirichlet nodes).
 * Replaces the context's load. Returns SOS_ENOCONV like sos_solve (outputs
 * still written). */
int sos_adjoint(sos_ctx* ctx, const double* dJ_dphi_nodes, double tol, double* dJ_ddrho_elem,
                double* psi_nodes, sos_stats* stats);

/* Search of transmission coefficients with CMA-ES (Sec. 4): minimises the
 * maximum over k in [kmin, kmax] (n_k uniform samples) of the two-subdomain
 * Fourier convergence factor (Sec. 3)
 *   rho(k) = |(k - L1)(k - L2)| / ((k + L1)(k + L2)),  L_s = p_s + q_s k^2
 * (the second-order operator read with the symbol p + q k^2).
 * kind: 0 zeroth order symmetric (p), 1 zeroth order unsymmetric (p1, p2),
 *       2 second order symmetric (p, q), 3 second order unsymmetric
 *       (p1, q1, p2, q2).
 * popsize: samples per generation (the paper uses 25); stops after max_iter
 * generations (the paper: 7200) or when the search distribution's spread or
 * the best cost's progress falls below tol (the paper: 5e-11).
 * Host memory, CPU only (no GPU needed): pq_out[4] = p1, q1, p2, q2 of the best
 * point, rho_out = its cost, iters_out (may be NULL) = generations run.
 * Deterministic for a seed. SOS_EINVAL on bad arguments. */
int sos_optimize_robin(int32_t kind, double kmin, double kmax, int32_t n_k, int32_t popsize, int32_t max_iter,
                       double tol, uint64_t seed, double* pq_out, double* rho_out, int32_t* iters_out);

/* Diagnostics used by the parity tests. */
/* y_s = A_s x_s for every subdomain s (concatenated local layout, device).
 * precision selects the FP64 (x, y double*) or FP32 (float*) operator. */
int sos_apply_local(sos_ctx* ctx, int32_t precision, const void* x, void* y);
/* Copy the outer state out of / into the context: u (local layout, FP64) and
 * lambda (face_off layout, FP64). Either pointer may be NULL. */
int sos_get_state(sos_ctx* ctx, double* u_local, double* lambda);
int sos_set_state(sos_ctx* ctx, const double* u_local, const double* lambda);
/* Load f_s from drho (as sos_solve) without iterating. */
int sos_set_density(sos_ctx* ctx, const double* drho_elem);
/* Run n outer iterations from the current state with the current load. */
int sos_iterate(sos_ctx* ctx, int32_t n, sos_stats* stats);
/* Global relative residual and glued solution of the current state. */
int sos_residual(sos_ctx* ctx, double* phi_nodes, double* rel_residual);
/* sos_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same global residual (and, if phi_nodes != NULL, the glued solution),
 * with its working vectors (the averaged copies, the local residuals, the
 * block partials, the result words) in a fixed scratch array of 48 MiB per
 * GPU that the library holds from its first set-up on that GPU until the
 * process ends, instead of the context's workspaces. Calls no allocating
 * routine. Contexts of more than about 3.1 M local unknowns (2 FP64 vectors
 * plus partials beyond 48 MiB) return SOS_EINVAL. Every context on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU race (the
 * library serialises nothing); a call overwrites every scratch value it reads,
 * so no clearing is needed. Host output rel_residual as sos_residual. */
int sos_residual_noalloc(sos_ctx* ctx, double* phi_nodes, double* rel_residual);
/* Residual history (Sec. 6 stops on the global residual): the outer
 * iteration count and relative residual of every convergence check since the
 * last solve started (or sos_set_state); sos_iterate appends. *n receives the
 * number of checks; the first min(cap, *n) are copied to outer / res (host
 * memory, either may be NULL). SOS_LOG=1 in the environment also prints one
 * line per check on stderr. */
int sos_history(const sos_ctx* ctx, int32_t cap, int32_t* n, int32_t* outer, double* res);
/* Inner PCG iterations (Sec. 6) of every subdomain in the last outer
 * iteration, subdomain order of sos_layout, copy after copy. *n receives the
 * number of subdomains of all copies; the first min(cap, *n) counts are copied
 * to iters (host memory, may be NULL). Synchronises the context's stream. */
int sos_inner_iters(sos_ctx* ctx, int32_t cap, int32_t* n, int32_t* iters);
/* Failure-handling tests: spin_ticks bounds the team barrier's wait (wall
 * clock ticks at 100 MHz; 0 restores the default, about 1.3 s); tag_skew = 1
 * makes every member wait for a tag no member writes, so each team barrier
 * ends at that bound and the solve reports SOS_EBREAKDOWN (every kernel still
 * exits normally). tag_skew = 0 is normal operation. */
int sos_debug_barrier(sos_ctx* ctx, int64_t spin_ticks, int32_t tag_skew);

void sos_destroy(sos_ctx* ctx);
const char* sos_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SOS_H */
