// Host-side launch wrappers of the HIP kernels (defined in sos_kernels.hip).
#pragma once

#include "sos_internal.h"

namespace sos {

// A block of a segmented launch: subdomain s, z-range [z0, z1) of its planes.
struct BlockDesc {
  int32_t s, z0, z1, pad;
};

// Launch geometry of a segmented launch (one block per BlockDesc).
struct SegLaunch {
  const BlockDesc* blocks;  // device
  const int32_t* bfirst;    // device, n_sub+1: blocks of s are [bfirst[s], bfirst[s+1])
  int32_t nblocks;
  int32_t threads;          // threads per block (multiple of 64)
  int32_t cpt;              // x-y columns per thread (1 to 4)
  size_t lds64;             // dynamic LDS bytes for FP64 marches
  size_t lds32;             // dynamic LDS bytes for FP32 marches
  int32_t zu;               // every block marches one segment (uniform-z residual)
};

struct Dev {
  const SubDesc* subs;      // device descriptors
  const FaceDesc* faces;
  Geom geo;
  int32_t n_faces;
  int32_t hasq;             // some face has a second-order coefficient q > 0
};

constexpr int kMaxTeam = 8;  // blocks per subdomain in the fused kernel
constexpr int kMinSeg = 8;  // shortest z-segment of a march (planes)

// Number of z-segments a block of `threads` threads with `cpt` x-y columns per
// thread marches at once over a z-range of zlen planes of an nx*ny plane.
__host__ __device__ inline int march_segments(int nx, int ny, int zlen, int threads, int cpt) {
  int S = nx * ny;
  int g = (threads * cpt) / S;
  int gz = (zlen + kMinSeg - 1) / kMinSeg;
  if (g > gz) g = gz;
  return g < 1 ? 1 : g;
}
// Wave-owned rows: wave w of a block owns the x-rows [w R, (w + 1) R) of the
// plane, R = ra_rows(nx, cpt) = floor(64 cpt / nx), so the x-pass of the
// operator reads only LDS values its own wave wrote and needs no workgroup
// barrier. Waves needed: ceil(ny / R); 0 when a row does not fit one wave.
__host__ __device__ inline int ra_rows(int nx, int cpt) { return (64 * cpt) / nx; }
__host__ __device__ inline int ra_waves(int nx, int ny, int cpt) {
  const int R = ra_rows(nx, cpt);
  return R < 1 ? 0 : (ny + R - 1) / R;
}
// LDS planes per march segment: the operand (a second one alternating by step
// where second-order terms or wave-owned rows need it) and the two y-pass
// results, each zero-padded by kPad; segments are kPlanes planes apart.
constexpr int kPlanes = 4;
// LDS planes a single-segment march uses: the second operand plane only with
// second-order face terms or wave-owned rows.
__host__ __device__ inline int march_planes(bool q, bool rows) { return (q || rows) ? kPlanes : kPlanes - 1; }
// LDS bytes of such a march.
__host__ __device__ inline size_t march_lds_bytes(int nx, int ny, int zlen, int threads, int cpt,
                                                  size_t elem) {
  size_t sp = (size_t)(nx + 2 * kPad) * (size_t)(ny + 2 * kPad);
  return kPlanes * sp * (size_t)march_segments(nx, ny, zlen, threads, cpt) * elem;
}

// f_s from a per-element density (FP64), for all subdomains.
hipError_t launch_load_density(const Dev& d, int max_n, const double* drho, double G,
                               double* f_loc, hipStream_t st);
// f_s = f_nodes / multiplicity.
hipError_t launch_load_nodes(const Dev& d, int max_n, const double* f_nodes, double* f_loc,
                             hipStream_t st);
// b = f + sum_j R_sj^T lambda_{s<-j} rewritten at the edge and corner nodes
// of the boundary shell (the exchange writes the other face nodes; inside,
// b = f), in bx on the x-boundary nodes (SubDesc::xoff) and in b elsewhere;
// then r = b - A u (FP64 apply), stored as Tr; partials (r'D^-1 r if rz, else
// 0), r'r, b'b per block. team_part (optional): the fused kernel's team
// slots, n_sub * kMaxTeam * 8 doubles, cleared for the launch that follows.
hipError_t launch_residual(const Dev& d, const SegLaunch& L, int fp32, bool rz, const double* u,
                           const double* f, const double* lam, double* b, double* bx, void* r_out, double* part,
                           double* team_part, hipStream_t st);
// Why a subdomain's inner solve stopped early, OR-ed into one device word
// per solve (the host reads it at every convergence check).
enum BreakBits : int32_t {
  kBrkCurvature = 1,   // non-positive p'Ap (or delta - beta gamma / alpha) in a CG
  kBrkNonFinite = 2,   // a non-finite residual, dot product or step length
  kBrkBarrier = 4,     // a team member gave up waiting at the team barrier
  kBrkLaunch = 8,      // the launch does not fit the kernel variant (host error)
};

// Per-subdomain CG scalars from the residual partials (stepwise path).
hipError_t launch_cg_init(const Dev& d, const SegLaunch& L, const double* part, double tol_rel,
                          double tol_abs, CgScal* scal, int32_t* ndone, hipStream_t st);
// Stepwise CG, iteration t: p <- D^-1 r + beta p ; q = A p ; partial p'q.
hipError_t launch_cg_apply(const Dev& d, const SegLaunch& L, int fp32, int t, int max_inner,
                           const void* r, const void* p_old, void* p_new, void* q, double* part,
                           CgScal* scal, int32_t* ndone, unsigned long long* counters, int32_t* flags,
                           hipStream_t st);
// Stepwise CG, iteration t: x += alpha p ; r -= alpha q ; partials r'z, r'r.
hipError_t launch_cg_update(const Dev& d, const SegLaunch& L, int fp32, int t, void* x, const void* p,
                            void* r, const void* q, double* part, CgScal* scal, int32_t* ndone,
                            int32_t* flags, hipStream_t st);
// u += x for every subdomain whose inner solve took at least one iteration and
// did not break down.
hipError_t launch_add_correction(const Dev& d, const SegLaunch& L, int fp32, double* u, const void* x,
                                 const CgScal* scal, hipStream_t st);
// Member tau of the team of T blocks that solves subdomain s (s < 0: an idle
// block that exits at once, padding the grid so that a team's members share
// blockIdx % 8, i.e. one XCD under round-robin dispatch).
struct TeamSlot {
  int32_t s, tau, T, pad;
};
// The fused inner solve: every block of the grid (fmap gives the block ->
// (subdomain, member) map, larger subdomains first) runs its part of a whole CG
// and adds the correction to u.
struct FusedArgs {
  const TeamSlot* fmap;    // nblocks entries
  const double* res_part;  // residual partials (segmented launch L)
  double tol_rel, tol_abs;
  int32_t max_inner;
  void *r, *r1, *w0, *w1, *s0, *s1, *p0, *p1, *x;  // CG vectors (r = the initial residual)
  double* u;
  CgScal* scal;
  unsigned long long* iters_total;  // [0] CG iterations, [1] algorithmic bytes
  int32_t nblocks;                  // grid size (teams plus idle padding blocks)
  int32_t team;                     // the largest team (1: no inter-block sync anywhere)
  double* team_part;                // n_sub * kMaxTeam * 2 * 4 tagged partial sums (cleared by
                                    // the residual kernel before each launch)
  int32_t zu;                       // every block marches one segment (uniform z variant)
  int32_t rows;                     // wave-owned rows (see ra_rows): one barrier per plane
  int32_t res;                      // resident in LDS (FP32, uniform z only): 1 p and x, 2 x
  uint32_t lds_bytes;               // dynamic LDS of the launch (march planes + resident p, x)
  int32_t* flags;                   // BreakBits of the solve, OR-ed by every block that stops early
  uint64_t spin_ticks;              // team barrier: longest wait (wall clock ticks, 100 MHz)
  int32_t tag_skew;                 // team barrier: 0; 1 waits for a tag no member writes, so
                                    // every wait ends at spin_ticks (failure-handling tests)
};
// lds: the march planes; with a.res the launch takes a.lds_bytes (march planes
// and the resident p and x of the largest z-range, at least lds). A team
// launch is a plain one when the kernel's occupancy admits the whole grid,
// else cooperative. plain != NULL: launch nothing, report whether the launch
// would be plain (and so can be captured in a graph).
hipError_t launch_fused_cg(const Dev& d, const SegLaunch& L, int fp32, int threads, int cpt, size_t lds,
                           const FusedArgs& a, hipStream_t st, bool* plain = nullptr);
// Robin exchange over all interfaces (in place, both directions).
// One interface pair (s <- j, j <- s) resolved on the host: where each side's
// face nodes sit in the local vectors (node (a, b) at base + a sa + b sb, a
// fastest), both lambda offsets, the summed coefficients and the tangential
// 1D rows (shared by both sides).
struct ExPair {
  int64_t base_s, sa_s, sb_s, base_j, sa_j, sb_j;
  // a side whose face is normal to its local axis 0 keeps its right-hand side
  // in the x-boundary array (SubDesc::xoff): base and strides there, else -1
  int64_t xb_s, xsa_s, xsb_s, xb_j, xsa_j, xsb_j;
  int64_t lam_f, lam_g;  // lambda_{s<-j}, lambda_{j<-s}
  double cp, cq;         // p_sj + p_js, q_sj + q_js
  double msa, msb, ksa, ksb;
  int32_t kla, klb, nea, neb, na, nb;
};
constexpr int kExchangeRows = 16;  // most face rows per block of the exchange kernel
constexpr int kExThreads = 512;    // threads of an exchange block
// Face rows per exchange block: as many as one pass of the block covers.
inline int exchange_rows(int max_na) {
  const int r = kExThreads / (max_na > 0 ? max_na : 1);
  return r < 1 ? 1 : (r > kExchangeRows ? kExchangeRows : r);
}
// Fused kernel block table (one block per subdomain) ordered by the work of
// each subdomain's last inner solve, longest first.
hipError_t launch_order_blocks(const Dev& d, const CgScal* scal, TeamSlot* fmap, hipStream_t st);
// Robin exchange of every interface pair; with b (and f) given, also
// b = f + lambda at both sides' face nodes (edge and corner nodes are left to
// the residual kernel); with fmap (and d, scal) given, the block ordering of
// launch_order_blocks runs as one more workgroup of it.
hipError_t launch_exchange(const ExPair* pairs, int32_t n_pairs, int32_t max_na, int32_t max_nb, const double* u,
                           double* lam, const double* f, double* b, const double* fx, double* bx, hipStream_t st,
                           const Dev* d = nullptr, const CgScal* scal = nullptr, TeamSlot* fmap = nullptr);
// b = f + sum_j R^T lambda on every shell node of the segmented launch's
// blocks, and fx, bx (f and b on the x-boundary nodes, SubDesc::xoff) (the
// start of a run: the residual kernel itself rewrites only edges and corners,
// the exchange the rest).
hipError_t launch_shell_rhs(const Dev& d, const SegLaunch& L, const double* f, const double* lam, double* b,
                            double* fx, double* bx, hipStream_t st);
// Global residual check. First pass: ut <- the average of each shell node's
// copies (local layout; interior entries untouched).
hipError_t launch_glue_shell(const Dev& d, int max_shell, const double* u, double* ut, hipStream_t st);
// Second pass (segmented launch L): rho = f - K^N u~ (FP64, local stiffness
// without Robin terms), u~ = ut on the shell and u inside; interior nodes add
// rho^2, f^2 to the block partials part[0 .. L.nblocks), shell nodes store
// rho; phi (if not null) <- u~ on owned nodes.
hipError_t launch_check_residual(const Dev& d, const SegLaunch& L, const double* u, const double* ut,
                                 const double* f, double* rho, double* phi, double* part, hipStream_t st);
// Shell nodes of a subdomain of n0 x n1 x n2 nodes: with at least 3 along
// every axis, the first and last planes, then the ring of each plane in
// between; with at most 2 along some axis, every node.
__host__ __device__ inline int shell_nodes(int n0, int n1, int n2) {
  if (n0 <= 2 || n1 <= 2 || n2 <= 2) return n0 * n1 * n2;
  return 2 * n0 * n1 + (n2 - 2) * (2 * (n0 + n1) - 4);
}
// Third pass: owned shell nodes, rho and f summed over copies; partials
// part[0 .. shell_blocks(d, max_shell)).
hipError_t launch_assemble_shell(const Dev& d, int max_shell, const double* rho, const double* f, double* part,
                                 hipStream_t st);
int shell_blocks(const Dev& d, int max_shell);
// Per copy res_c = sqrt(sum rr / sum ff) over both passes' partials (na of the
// first, then nb of the second) -> dev_out[3 + c]; the largest over the
// copies -> dev_out[0] and host_out[0] (host-mapped, may be null); the solve's
// BreakBits (flags, may be null) -> host_out[1].
hipError_t launch_final_norm(const double* part, int32_t na, int32_t nb, int32_t copies, const int32_t* flags,
                             double* dev_out, double* host_out, hipStream_t st);
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t st);
// grad_e = 4 pi G sum_a psi_a int_e phi_a for every element (psi over all nodes).
hipError_t launch_grad_density(const Geom& g, const double* psi, double G, double* grad, hipStream_t st);
// y = A x (diagnostic; fp32 selects float vectors).
hipError_t launch_apply(const Dev& d, const SegLaunch& L, int fp32, const void* x, void* y,
                        hipStream_t st);

constexpr int kAssembleThreads = 256;

// Largest block the kernels are compiled for with `cpt` x-y columns per thread.
int launch_bound(int cpt);

}  // namespace sos
