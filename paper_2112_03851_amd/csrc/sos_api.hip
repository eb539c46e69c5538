// C-ABI of the Robin-Schwarz subdomain-solve library: validation, descriptors,
// workspaces, the outer iteration (Sec. 3) and its convergence check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <sys/stat.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/sos.h"
#include "sos_internal.h"
#include "sos_kernels.h"

using namespace sos;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(SOS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

struct Seg {
  std::vector<BlockDesc> blocks;
  std::vector<int32_t> bfirst;
  BlockDesc* d_blocks = nullptr;
  int32_t* d_bfirst = nullptr;
  SegLaunch L{};
};

// Scratch memory of the allocation-free entry points: one array per GPU, in
// device memory from the moment the library's code object is loaded on that
// GPU until the process ends. Host code never uses the name `scratch` as an
// address (it is a host-side stand-in there); it uses the device address that
// hipGetSymbolAddress returns, resolved once per device at set-up.
constexpr size_t kScratchBytes = size_t(48) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on first use
// per device, with that device current).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SOS_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(SOS_ESTATE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(SOS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SOS_OK;
}

}  // namespace

struct sos_ctx {
  sos_mesh mesh{};
  sos_opts opts{};
  int fp32 = 0;
  Geom geo{};
  std::vector<SubDesc> subs;
  std::vector<FaceDesc> faces;
  std::vector<int32_t> pairs;
  std::vector<int32_t> order;
  int64_t n_local = 0, n_lam = 0, n_nodes = 0;
  int max_n = 0, max_face = 0, max_face_na = 0, max_face_nb = 0;
  Dev dev{};
  SubDesc* d_subs = nullptr;
  FaceDesc* d_faces = nullptr;
  ExPair* d_expairs = nullptr;  // the pairs resolved for the exchange kernel
  // fused kernel: team size per subdomain, its size bucket (0 = largest), and
  // the block -> (subdomain, member) table
  std::vector<int32_t> sub_team, sub_bucket;
  int n_buckets = 1;
  std::vector<TeamSlot> fmap;
  TeamSlot* d_fmap = nullptr;
  size_t fmap_cap = 0;
  bool fmap_dirty = true;
  Seg seg;
  // workspaces
  double *u = nullptr, *f = nullptr, *lam = nullptr, *ut = nullptr, *rho = nullptr;
  double* b = nullptr;  // local right-hand side f_s + sum_j R_sj^T lambda_{s<-j}
  // f and b on the x-boundary nodes (i = 0, n0 - 1) of every subdomain,
  // contiguous per face (SubDesc::xoff); b there is not used
  double *fxf = nullptr, *bxf = nullptr;
  int64_t n_xface = 0;
  void *r = nullptr, *x = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
  void *r1 = nullptr, *w1 = nullptr, *s0 = nullptr, *s1 = nullptr;  // fused CG only
  double* part = nullptr;       // 3 per segmented block
  double* part_norm = nullptr;  // 2 per assemble block
  int max_shell = 0;     // most shell nodes of a subdomain
  int n_norm_blocks = 0;  // residual check partials: march blocks, then shell blocks
  double* d_res = nullptr;      // [res, r'r, f'f]
  double* psi = nullptr;        // adjoint field over all nodes (allocated on first use)
  CgScal* scal = nullptr;
  int32_t* ndone = nullptr;
  unsigned long long* counters = nullptr;  // [0] inner iterations, [1] algorithmic bytes
  int32_t* flags = nullptr;                // BreakBits of the current solve (device word)
  double* h_res = nullptr;                 // pinned, coherent, device-mapped: [residual, flags]
  double* d_hres = nullptr;                // device view of h_res
  int32_t* h_ndone = nullptr;              // pinned
  unsigned long long* h_counters = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // fused kernel launch shape
  int fused_threads = 0, fused_cpt = 1, fused_team = 1;
  int fused_ra = 0;   // wave-owned rows in the fused kernel
  int fused_res = 0;  // p and x resident in LDS when they fit (FP32, uniform z)
  size_t fused_lds = 0;
  double* team_part = nullptr;   // team partial sums
  bool tuned = false;    // fused block shape chosen (explicit or autotuned)
  double tune_ms = 0.0;  // duration of the chosen shape in the tuning run
  size_t lds_limit = 0;
  // graph of (check_every outer iterations + check)
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_k = 0;
  std::vector<hipEvent_t> gevents;
  // timing
  double kernel_ms = 0.0;
  int64_t kernel_launches = 0;
  bool have_load = false;
  // team barrier wait bound and tag skew (sos_debug_barrier)
  uint64_t spin_ticks = 1ull << 27;
  int32_t tag_skew = 0;
  void* scratch = nullptr;  // device address of this device's scratch array
  // (outer iteration, relative residual) of every check since the last solve start
  std::vector<int32_t> hist_outer;
  std::vector<double> hist_res;
  int32_t outer_total = 0;
};

namespace {

int64_t align64(int64_t v) { return (v + 63) & ~int64_t(63); }

constexpr int kStallOuter = 2000;  // outer iterations without 1% progress
constexpr int kMaxCopies = 4096;   // independent problem copies of one context

void release(sos_ctx* c) {
  if (!c) return;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  for (auto e : c->gevents) (void)hipEventDestroy(e);
  void* ptrs[] = {c->d_subs, c->d_faces, c->d_expairs, c->d_fmap, c->seg.d_blocks, c->seg.d_bfirst, c->u, c->f, c->b,
                  c->fxf, c->bxf,
                  c->lam, c->ut, c->rho, c->r, c->x, c->p0, c->p1, c->q, c->r1, c->w1, c->s0, c->s1,
                  c->part, c->part_norm, c->d_res, c->psi, c->team_part,
                  c->scal, c->ndone, c->counters, c->flags};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_res) (void)hipHostFree(c->h_res);
  if (c->h_ndone) (void)hipHostFree(c->h_ndone);
  if (c->h_counters) (void)hipHostFree(c->h_counters);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

void invalidate_graph(sos_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->graph_k = 0;
  for (auto e : c->gevents) (void)hipEventDestroy(e);
  c->gevents.clear();
}

int check_opts(const sos_opts* o) {
  if (o->precision != SOS_FP64 && o->precision != SOS_FP32_INNER) return fail(SOS_EINVAL, "opts.precision must be SOS_FP64 or SOS_FP32_INNER");
  if (o->mode != SOS_STEPWISE && o->mode != SOS_BATCHED) return fail(SOS_EINVAL, "opts.mode must be SOS_STEPWISE or SOS_BATCHED");
  if (o->max_outer < 1) return fail(SOS_EINVAL, "opts.max_outer must be >= 1");
  if (o->max_inner < 1) return fail(SOS_EINVAL, "opts.max_inner must be >= 1");
  if (o->check_every < 1) return fail(SOS_EINVAL, "opts.check_every must be >= 1");
  if (!(o->inner_tol >= 0.0) || !(o->inner_abs >= 0.0) || (o->inner_tol == 0.0 && o->inner_abs == 0.0))
    return fail(SOS_EINVAL, "opts.inner_tol/inner_abs must be >= 0 and not both 0");
  if (!(o->G > 0.0) || !std::isfinite(o->G)) return fail(SOS_EINVAL, "opts.G must be positive");
  if (o->block != 0 && (o->block < 64 || o->block > 1024 || o->block % 64))
    return fail(SOS_EINVAL, "opts.block must be 0 or a multiple of 64 in [64, 1024]");
  if (o->team < 0 || o->team > kMaxTeam) return fail(SOS_EINVAL, "opts.team must be in [0, %d]", kMaxTeam);
  if (o->wave_rows != 0 && o->wave_rows != 1) return fail(SOS_EINVAL, "opts.wave_rows must be 0 or 1");
  if (o->wave_rows && !o->block) return fail(SOS_EINVAL, "opts.wave_rows needs opts.block");
  if (o->resident != 0 && o->resident != 1) return fail(SOS_EINVAL, "opts.resident must be 0 or 1");
  if (o->march < 0 || o->march > 3) return fail(SOS_EINVAL, "opts.march must be 0 (automatic), 1, 2 or 3");
  if (o->schedule != 0 && o->schedule != 1) return fail(SOS_EINVAL, "opts.schedule must be 0 or 1");
  return SOS_OK;
}

int apply_robin(sos_ctx* c, const sos_robin* rb) {
  if (!rb) return fail(SOS_EINVAL, "robin is NULL");
  if (rb->order != 0 && rb->order != 2) return fail(SOS_EINVAL, "robin.order must be 0 or 2");
  std::vector<double> pv(c->faces.size()), qv(c->faces.size(), 0.0);
  for (size_t f = 0; f < c->faces.size(); ++f) {
    double p = rb->p ? rb->p[f] : rb->p0;
    if (!(p > 0.0) || !std::isfinite(p)) return fail(SOS_EINVAL, "Robin coefficient of face %zu must be > 0", f);
    pv[f] = p;
    if (rb->order == 2) {
      double q = rb->q ? rb->q[f] : rb->q0;
      if (!(q >= 0.0) || !std::isfinite(q)) return fail(SOS_EINVAL, "second-order coefficient of face %zu must be >= 0", f);
      qv[f] = q;
    }
  }
  c->dev.hasq = 0;
  for (size_t f = 0; f < c->faces.size(); ++f) {
    c->faces[f].p = pv[f];
    c->faces[f].q = qv[f];
    if (qv[f] > 0.0) c->dev.hasq = 1;
  }
  for (auto& s : c->subs) {
    for (int a = 0; a < 3; ++a) {
      s.elo[a] = s.face[2 * a] >= 0 ? c->faces[s.face[2 * a]].p : 0.0;
      s.ehi[a] = s.face[2 * a + 1] >= 0 ? c->faces[s.face[2 * a + 1]].p : 0.0;
      s.qlo[a] = s.face[2 * a] >= 0 ? c->faces[s.face[2 * a]].q : 0.0;
      s.qhi[a] = s.face[2 * a + 1] >= 0 ? c->faces[s.face[2 * a + 1]].q : 0.0;
    }
  }
  return SOS_OK;
}

// Segmented launch: each subdomain's z-range split into chunks so that the
// grid has several blocks per compute unit.
int build_seg(sos_ctx* c) {
  Seg& g = c->seg;
  int smax = 0;
  for (auto& s : c->subs) smax = std::max(smax, s.n[0] * s.n[1]);
  int cpt = 1;
  while (cpt < 4 && (smax + cpt - 1) / cpt > 1024) cpt *= 2;
  // FP64 contexts (the stepwise form's apply and update, its residual): two
  // columns per thread means nine or more waves per block, held to 168 VGPRs,
  // where the FP64 marches spill; three columns fit 512 threads with 256 VGPRs
  // and none (39.4 against 43.1 ms per outer iteration on 128^3)
  if (!c->fp32 && cpt == 2 && (smax + 2) / 3 <= 512) cpt = 3;
  if ((smax + cpt - 1) / cpt > 1024) return fail(SOS_EINVAL, "x-y plane of %d nodes exceeds the supported maximum", smax);
  int threads = ((smax + cpt - 1) / cpt + 63) / 64 * 64;
  const int n_sub = (int)c->subs.size();
  const int want = std::max(1, (2 * 256 + n_sub - 1) / n_sub);
  g.blocks.clear();
  g.bfirst.assign(1, 0);
  size_t lds64 = 0, lds32 = 0;
  bool zu = true;
  for (int s = 0; s < n_sub; ++s) {
    const SubDesc& d = c->subs[s];
    const int nz = d.n[2];
    int chunks = std::min(want, std::max(1, nz / kMinSeg));
    int len = (nz + chunks - 1) / chunks;
    for (int z = 0; z < nz; z += len) {
      BlockDesc b{s, z, std::min(nz, z + len), 0};
      g.blocks.push_back(b);
      zu = zu && march_segments(d.n[0], d.n[1], b.z1 - b.z0, threads, cpt) == 1;
      lds64 = std::max(lds64, march_lds_bytes(d.n[0], d.n[1], b.z1 - b.z0, threads, cpt, 8));
      lds32 = std::max(lds32, march_lds_bytes(d.n[0], d.n[1], b.z1 - b.z0, threads, cpt, 4));
    }
    g.bfirst.push_back((int32_t)g.blocks.size());
  }
  if (lds64 > c->lds_limit) return fail(SOS_EINVAL, "subdomain plane needs %zu bytes of LDS (limit %zu)", lds64, c->lds_limit);
  g.L.nblocks = (int32_t)g.blocks.size();
  g.L.threads = threads;
  g.L.cpt = cpt;
  g.L.lds64 = lds64;
  g.L.lds32 = lds32;
  g.L.zu = zu ? 1 : 0;
  return SOS_OK;
}

int smax_plane(const sos_ctx* c) {
  int smax = 0;
  for (auto& s : c->subs) smax = std::max(smax, s.n[0] * s.n[1]);
  return smax;
}

size_t fused_lds_need(const sos_ctx* c, int threads, int cpt) {
  size_t es = c->fp32 ? 4 : 8, lds = 0;
  for (auto& s : c->subs) lds = std::max(lds, march_lds_bytes(s.n[0], s.n[1], s.n[2], threads, cpt, es));
  return lds;
}

// Sets the fused kernel's block shape; cpt = 0 picks the fewest columns per
// thread that cover the largest x-y plane.
int fused_shape(sos_ctx* c, int threads, int cpt = 0, int ra = 0, int res = 0) {
  const int smax = smax_plane(c);
  if (threads == 0) {
    int k = 1;
    while (k < 4 && (smax + k - 1) / k > 1024) k *= 2;
    threads = std::max(((smax + k - 1) / k + 63) / 64 * 64, 256);
  }
  if (cpt == 0) {
    cpt = 1;
    while (cpt < 4 && cpt * threads < smax) ++cpt;
  }
  if (cpt * threads < smax) return fail(SOS_EINVAL, "block of %d threads cannot cover a %d-node plane", threads, smax);
  if (threads > launch_bound(cpt))
    return fail(SOS_EINVAL, "block of %d threads with %d columns each exceeds the kernel bound %d", threads, cpt,
                launch_bound(cpt));
  const size_t lds = fused_lds_need(c, threads, cpt);
  if (lds > c->lds_limit) return fail(SOS_EINVAL, "fused kernel needs %zu bytes of LDS (limit %zu)", lds, c->lds_limit);
  if (ra) {
    if (threads % 64) return fail(SOS_EINVAL, "wave-owned rows need a multiple of 64 threads");
    for (auto& s : c->subs) {
      const int w = ra_waves(s.n[0], s.n[1], cpt);
      if (w < 1 || w > threads / 64)
        return fail(SOS_EINVAL, "wave-owned rows: %d waves of %d columns cannot cover a %dx%d plane", threads / 64,
                    64 * cpt, s.n[0], s.n[1]);
    }
  }
  c->fused_threads = threads;
  c->fused_cpt = cpt;
  c->fused_ra = ra ? 1 : 0;
  c->fused_res = res ? 1 : 0;
  c->fused_lds = lds;
  return SOS_OK;
}

// True when every block of the fused kernel (every subdomain and team member)
// marches a single segment, so the uniform-z kernel variant applies.
bool fused_one_segment(const sos_ctx* c) {
  if (c->fused_ra) return true;  // wave-owned rows: one segment by construction
  for (size_t i = 0; i < c->subs.size(); ++i) {
    const SubDesc& s = c->subs[i];
    const int T = c->sub_team[i];
    for (int tau = 0; tau < T; ++tau) {
      const int zlen = ((tau + 1) * s.n[2]) / T - (tau * s.n[2]) / T;
      if (march_segments(s.n[0], s.n[1], zlen, c->fused_threads, c->fused_cpt) != 1) return false;
    }
  }
  return true;
}

// Team sizes per subdomain (every copy of a subdomain gets the same).
int set_teams(sos_ctx* c, const std::vector<int32_t>& teams) {
  if (teams.size() != c->subs.size()) return fail(SOS_EINVAL, "one team size per subdomain expected");
  int mx = 1;
  for (size_t i = 0; i < teams.size(); ++i) {
    const int t = teams[i];
    if (t < 1 || t > kMaxTeam) return fail(SOS_EINVAL, "team must be in [1, %d]", kMaxTeam);
    if (c->subs[i].n[2] < t)
      return fail(SOS_EINVAL, "team of %d blocks exceeds subdomain %zu's %d z-planes (marched planes)", t, i,
                  c->subs[i].n[2]);
    mx = std::max(mx, t);
  }
  c->sub_team = teams;
  c->fused_team = mx;
  c->fmap_dirty = true;
  invalidate_graph(c);
  return SOS_OK;
}

int set_team(sos_ctx* c, int team) { return set_teams(c, std::vector<int32_t>(c->subs.size(), team)); }

// One team size per size bucket (teams[b] for bucket b).
int set_bucket_teams(sos_ctx* c, const std::vector<int32_t>& teams) {
  std::vector<int32_t> t(c->subs.size());
  for (size_t i = 0; i < t.size(); ++i) t[i] = teams[c->sub_bucket[i]];
  return set_teams(c, t);
}

// Size buckets of the subdomains (0 = largest): one bucket when the node
// counts differ by at most 1.5x, else three of equal width in log size.
void make_buckets(sos_ctx* c) {
  int64_t lo = INT64_MAX, hi = 0;
  std::vector<int64_t> n(c->subs.size());
  for (size_t i = 0; i < n.size(); ++i) {
    n[i] = (int64_t)c->subs[i].n[0] * c->subs[i].n[1] * c->subs[i].n[2];
    lo = std::min(lo, n[i]);
    hi = std::max(hi, n[i]);
  }
  c->sub_bucket.assign(n.size(), 0);
  c->n_buckets = 1;
  if (hi <= lo * 3 / 2) return;
  c->n_buckets = 3;
  const double span = std::log((double)hi / (double)lo);
  for (size_t i = 0; i < n.size(); ++i) {
    const int k = std::min(2, (int)(3.0 * std::log((double)n[i] / (double)lo) / span));
    c->sub_bucket[i] = 2 - k;
  }
}

// The fused kernel's block table: teams in the order of c->order (largest
// subdomain first). With a team of two or more blocks anywhere, the members of
// every team share blockIdx % 8 (one XCD under round-robin dispatch, so their
// halo planes and partials meet in one L2): each team goes to the shortest of
// eight queues and block b = 8 * position + queue, the queues padded with idle
// blocks. Uploaded before launches (never during a graph capture).
int ensure_fmap(sos_ctx* c) {
  if (!c->fmap_dirty) return SOS_OK;
  std::vector<TeamSlot>& m = c->fmap;
  m.clear();
  if (c->fused_team <= 1) {
    for (int32_t s : c->order) m.push_back({s, 0, 1, 0});
  } else {
    std::vector<std::vector<TeamSlot>> q(8);
    for (int32_t s : c->order) {
      size_t best = 0;
      for (size_t k = 1; k < q.size(); ++k)
        if (q[k].size() < q[best].size()) best = k;
      const int T = c->sub_team[s];
      for (int tau = 0; tau < T; ++tau) q[best].push_back({s, tau, T, 0});
    }
    size_t len = 0;
    for (auto& v : q) len = std::max(len, v.size());
    m.assign(8 * len, TeamSlot{-1, 0, 1, 0});
    for (size_t k = 0; k < q.size(); ++k)
      for (size_t i = 0; i < q[k].size(); ++i) m[8 * i + k] = q[k][i];
  }
  if (m.size() > c->fmap_cap) return fail(SOS_EINVAL, "fused block table of %zu entries exceeds %zu", m.size(), c->fmap_cap);
  HIPCHK(hipMemcpy(c->d_fmap, m.data(), m.size() * sizeof(TeamSlot), hipMemcpyHostToDevice));
  c->fmap_dirty = false;
  return SOS_OK;
}

struct Shape {
  int threads, cpt, ra, res;
  bool operator==(const Shape& o) const {
    return threads == o.threads && cpt == o.cpt && ra == o.ra && res == o.res;
  }
};

// Candidate block shapes of the fused kernel: for 1..4 columns per thread,
// the smallest block covering the largest plane and 1.5x, 2x, 3x that size
// (more segments per block on small planes), and the block of wave-owned rows,
// within the kernel bounds and LDS.
std::vector<Shape> fused_candidates(const sos_ctx* c) {
  const int smax = smax_plane(c);
  std::vector<Shape> out;
  auto add = [&](Shape sh) {
    if (sh.threads > launch_bound(sh.cpt) || fused_lds_need(c, sh.threads, sh.cpt) > c->lds_limit) return;
    if (std::find(out.begin(), out.end(), sh) == out.end()) out.push_back(sh);
  };
  for (int cpt = 1; cpt <= 4; ++cpt) {
    const int tmin = std::max(64, ((smax + cpt - 1) / cpt + 63) / 64 * 64);
    std::vector<int> sizes = {tmin, tmin + 64, tmin + 128};
    for (int mul2 : {3, 4, 6}) sizes.push_back((tmin * mul2 / 2 + 63) / 64 * 64);
    for (int t : sizes) add({t, cpt, 0, 0});
    int waves = 0;
    for (auto& s : c->subs) {
      const int w = ra_waves(s.n[0], s.n[1], cpt);
      waves = w < 1 ? 1 << 20 : std::max(waves, w);
    }
    if (waves <= 16) add({64 * waves, cpt, 1, 0});
  }
  // each shape again with p and x resident in LDS (used where they fit)
  if (c->fp32 && c->opts.resident) {
    const size_t n = out.size();
    for (size_t i = 0; i < n; ++i) out.push_back({out[i].threads, out[i].cpt, out[i].ra, 1});
  }
  // (shapes with res = 1 keep p and x in LDS, or x alone where both do not fit)
  return out;
}

// LDS bytes of a resident fused-kernel block (one segment): the march planes
// plus, per node of the largest z-range of a team member, `words` FP32 values
// (2: p and x, 1: x).
size_t fused_res_lds(const sos_ctx* c, int words) {
  size_t need = 0;
  const int planes = march_planes(c->dev.hasq != 0, c->fused_ra != 0);
  for (size_t i = 0; i < c->subs.size(); ++i) {
    const SubDesc& s = c->subs[i];
    const int T = c->sub_team[i];
    for (int tau = 0; tau < T; ++tau) {
      const size_t zlen = (size_t)(((tau + 1) * s.n[2]) / T - (tau * s.n[2]) / T);
      const size_t sp = (size_t)(s.n[0] + 2 * kPad) * (size_t)(s.n[1] + 2 * kPad);
      need = std::max(need, (planes * sp + words * zlen * (size_t)s.n[0] * (size_t)s.n[1]) * sizeof(float));
    }
  }
  return need;
}

std::string tune_key(const sos_ctx* c) {
  // geometry of the subdomain set, precision and inner tolerance
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  for (auto& s : c->subs)
    for (int a = 0; a < 3; ++a) mix((uint64_t)s.n[a]);
  mix((uint64_t)c->subs.size());
  char buf[160];
  snprintf(buf, sizeof buf, "gfx950|v3|%s|%016llx|tol%.3g|abs%.3g|max%d", c->fp32 ? "fp32" : "fp64",
           (unsigned long long)h, c->opts.inner_tol, c->opts.inner_abs, c->opts.max_inner);
  return buf;
}

std::string tune_cache_path() {
  const char* p = getenv("SOS_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/sos_autotune.jsonl";
}

// One cached tuning result: "teams" holds one team size per size bucket (an
// entry with a single "team" is a uniform team, one bucket).
bool tune_lookup(const std::string& key, int* threads, int* cpt, std::vector<int32_t>* teams, int* ra, int* res) {
  FILE* f = fopen(tune_cache_path().c_str(), "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (fgets(line, sizeof line, f)) {
    if (!strstr(line, pat.c_str())) continue;
    const char* t = strstr(line, "\"threads\": ");
    const char* k = strstr(line, "\"cpt\": ");
    const char* m = strstr(line, "\"teams\": [");
    if (!t || !k || !m || sscanf(t + 11, "%d", threads) != 1 || sscanf(k + 7, "%d", cpt) != 1) continue;
    std::vector<int32_t> tv;
    for (const char* q = m + 10; *q && *q != ']';) {
      char* e = nullptr;
      const long v = strtol(q, &e, 10);
      if (e == q) break;
      tv.push_back((int32_t)v);
      q = e;
      while (*q == ',' || *q == ' ') ++q;
    }
    if (tv.empty()) continue;
    found = true;
    *teams = tv;
    *ra = 0;
    *res = 0;
    const char* w = strstr(line, "\"rows\": ");
    if (w) (void)sscanf(w + 8, "%d", ra);
    const char* v = strstr(line, "\"resident\": ");
    if (v) (void)sscanf(v + 12, "%d", res);
  }
  fclose(f);
  return found;
}

void tune_store(const std::string& key, int threads, int cpt, const std::vector<int32_t>& teams, int ra, int res,
                double ms) {
  std::string path = tune_cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) mkdir(path.substr(0, slash).c_str(), 0755);
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  std::string tl;
  for (size_t i = 0; i < teams.size(); ++i) tl += (i ? ", " : "") + std::to_string(teams[i]);
  fprintf(f,
          "{\"key\": \"%s\", \"threads\": %d, \"cpt\": %d, \"teams\": [%s], \"rows\": %d, \"resident\": %d, "
          "\"ms\": %.4f}\n",
          key.c_str(), threads, cpt, tl.c_str(), ra, res, ms);
  fclose(f);
}

template <typename T>
int dalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return fail(SOS_ENOMEM, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
  return SOS_OK;
}

int dalloc_v(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e != hipSuccess) return fail(SOS_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  return SOS_OK;
}

// The local axis order of every subdomain (its descriptors are built in
// global order first). The marched axis is z unless the subdomain's x-y node
// plane holds more than kMaxPlane nodes, then the axis across the smallest
// node plane; march (1, 2, 3) forces x, y or z for every subdomain. The other
// two axes keep their global order (the lower one fastest).
void choose_axes(sos_ctx* c, int march) {
  for (auto& d : c->subs) {
    int m = 2;
    if (march) {
      m = march - 1;
    } else if ((int64_t)d.n[0] * d.n[1] > kMaxPlane) {
      int64_t best = INT64_MAX;
      for (int g = 2; g >= 0; --g) {
        const int64_t plane = (int64_t)d.n[(g + 1) % 3] * d.n[(g + 2) % 3];
        if (plane < best) {
          best = plane;
          m = g;
        }
      }
    }
    int perm[3], k = 0;
    for (int g = 0; g < 3; ++g)
      if (g != m) perm[k++] = g;
    perm[2] = m;
    const SubDesc o = d;
    for (int a = 0; a < 3; ++a) {
      const int g = perm[a];
      d.n[a] = o.n[g];
      d.klo[a] = o.klo[g];
      d.ne2[a] = o.ne2[g];
      d.face[2 * a] = o.face[2 * g];
      d.face[2 * a + 1] = o.face[2 * g + 1];
      d.perm[a] = g;
      d.iperm[g] = a;
      d.ks[a] = c->geo.ks[g];
      d.ms[a] = c->geo.ms[g];
    }
    // a face datum runs along its tangential axis of lower global index first
    d.tswap = 0;
    for (int a = 0; a < 3; ++a) {
      const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
      if (perm[t1] > perm[t2]) d.tswap |= 1 << a;
    }
    d.pad = 0;
  }
}

// The exchange kernel's pair descriptors from the host face and subdomain
// descriptors (again after every change of the Robin coefficients).
hipError_t upload_expairs(sos_ctx* c) {
  std::vector<ExPair> v;
  v.reserve(c->pairs.size());
  for (int32_t fi : c->pairs) {
    const FaceDesc& F = c->faces[fi];
    const FaceDesc& G = c->faces[F.opp];
    ExPair P{};
    const int ax = F.axis, ta = ax == 0 ? 1 : 0, tb = ax == 2 ? 1 : 2;
    // strides of the global axes in each side's local layout
    // and, for a face normal to the side's local axis 0, base and strides in
    // the x-boundary arrays (node (j, k) at xoff + side n1 n2 + j + n1 k;
    // one node thick: the i = 0 half)
    auto place = [&](const FaceDesc& X, int64_t* base, int64_t* sa, int64_t* sb, int64_t* xb, int64_t* xsa,
                     int64_t* xsb) {
      const SubDesc& sd = c->subs[X.s];
      const int64_t st[3] = {1, sd.n[0], (int64_t)sd.n[0] * sd.n[1]};
      *sa = st[sd.iperm[ta]];
      *sb = st[sd.iperm[tb]];
      const int la = sd.iperm[ax];
      *base = sd.off + (int64_t)(X.side ? sd.n[la] - 1 : 0) * st[la];
      *xb = *xsa = *xsb = -1;
      if (la == 0) {
        *xsa = *sa / sd.n[0];
        *xsb = *sb / sd.n[0];
        *xb = sd.xoff + ((X.side && sd.n[0] > 1) ? (int64_t)sd.n[1] * sd.n[2] : 0);
      }
    };
    place(F, &P.base_s, &P.sa_s, &P.sb_s, &P.xb_s, &P.xsa_s, &P.xsb_s);
    place(G, &P.base_j, &P.sa_j, &P.sb_j, &P.xb_j, &P.xsa_j, &P.xsb_j);
    const SubDesc& sd = c->subs[F.s];
    P.lam_f = F.lam_off;
    P.lam_g = G.lam_off;
    P.cp = F.p + G.p;
    P.cq = F.q + G.q;
    P.msa = c->geo.ms[ta];
    P.msb = c->geo.ms[tb];
    P.ksa = c->geo.ks[ta];
    P.ksb = c->geo.ks[tb];
    P.kla = sd.klo[sd.iperm[ta]];
    P.klb = sd.klo[sd.iperm[tb]];
    P.nea = sd.ne2[sd.iperm[ta]];
    P.neb = sd.ne2[sd.iperm[tb]];
    P.na = F.na;
    P.nb = F.nb;
    v.push_back(P);
  }
  if (v.empty()) return hipSuccess;
  return hipMemcpy(c->d_expairs, v.data(), v.size() * sizeof(ExPair), hipMemcpyHostToDevice);
}

// ------------------------------------------------------------------ outer iteration pieces

// The global residual check into the partials `part` (n_norm_blocks pairs)
// with ut and rho (local layout) as its working vectors.
int check_passes(sos_ctx* c, double* ut, double* rho, double* part, double* dres, double* phi) {
  hipStream_t st = c->stream;
  const int na = c->seg.L.nblocks;
  HIPCHK(launch_glue_shell(c->dev, c->max_shell, c->u, ut, st));
  HIPCHK(launch_check_residual(c->dev, c->seg.L, c->u, ut, c->f, rho, phi, part, st));
  HIPCHK(launch_assemble_shell(c->dev, c->max_shell, rho, c->f, part + 2 * (size_t)na, st));
  HIPCHK(launch_final_norm(part, na, c->n_norm_blocks - na, c->geo.copies, c->flags, dres, c->d_hres, st));
  return SOS_OK;
}

int enqueue_check(sos_ctx* c, double* phi) { return check_passes(c, c->ut, c->rho, c->part_norm, c->d_res, phi); }

FusedArgs fused_args(sos_ctx* c) {
  FusedArgs a;
  a.fmap = c->d_fmap;
  a.nblocks = (int32_t)c->fmap.size();
  a.res_part = c->part;
  a.tol_rel = c->opts.inner_tol;
  a.tol_abs = c->opts.inner_abs;
  a.max_inner = c->opts.max_inner;
  a.r = c->r;
  a.r1 = c->r1;
  a.w0 = c->q;
  a.w1 = c->w1;
  a.s0 = c->s0;
  a.s1 = c->s1;
  a.p0 = c->p0;
  a.p1 = c->p1;
  a.x = c->x;
  a.u = c->u;
  a.scal = c->scal;
  a.iters_total = c->counters;
  a.team = c->fused_team;
  a.team_part = c->team_part;
  a.zu = fused_one_segment(c) ? 1 : 0;
  a.rows = c->fused_ra;
  // resident p and x where they fit, else x alone, else neither
  a.res = 0;
  a.lds_bytes = (uint32_t)c->fused_lds;
  a.flags = c->flags;
  a.spin_ticks = c->spin_ticks;
  a.tag_skew = c->tag_skew;
  if (c->fused_res && c->fp32 && a.zu) {
    for (int words = 2; words >= 1 && !a.res; --words) {
      const size_t total = std::max(fused_res_lds(c, words), c->fused_lds);
      if (total <= c->lds_limit) {
        a.res = words == 2 ? 1 : 2;
        a.lds_bytes = (uint32_t)total;
      }
    }
  }
  return a;
}

// b = f on every node; a run starts by adding the Robin data on the boundary
// shell (b = f + sum_j R^T lambda there), then every exchange rewrites b at
// the face nodes and every residual at the edges and corners.
hipError_t copy_load_to_rhs(sos_ctx* c) {
  return hipMemcpyAsync(c->b, c->f, c->n_local * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
}

// One outer iteration in the batched form; ev (optional) brackets the fused kernel.
// With one block per subdomain, the fused kernel's next launch takes the
// subdomains in decreasing order of the work of their last inner solve.
bool schedule_by_work(const sos_ctx* c) {
  return c->opts.schedule && c->fused_team <= 1 && c->fmap.size() == c->subs.size();
}

int enqueue_batched_iteration(sos_ctx* c, hipEvent_t ev0, hipEvent_t ev1) {
  hipStream_t st = c->stream;
  HIPCHK(launch_residual(c->dev, c->seg.L, c->fp32, false, c->u, c->f, c->lam, c->b, c->bxf, c->r, c->part,
                         c->fused_team > 1 ? c->team_part : nullptr, st));
  if (ev0) HIPCHK(hipEventRecord(ev0, st));
  HIPCHK(launch_fused_cg(c->dev, c->seg.L, c->fp32, c->fused_threads, c->fused_cpt, c->fused_lds, fused_args(c), st));
  if (ev1) HIPCHK(hipEventRecord(ev1, st));
  // the block ordering runs inside the exchange launch (one more workgroup)
  const bool order = schedule_by_work(c);
  HIPCHK(launch_exchange(c->d_expairs, (int32_t)c->pairs.size(), c->max_face_na, c->max_face_nb, c->u, c->lam, c->f,
                         c->b, c->fxf, c->bxf, st, order ? &c->dev : nullptr, order ? c->scal : nullptr,
                         order ? c->d_fmap : nullptr));
  return SOS_OK;
}

// One outer iteration in the stepwise form (host-driven CG steps).
int stepwise_iteration(sos_ctx* c) {
  hipStream_t st = c->stream;
  const SegLaunch& L = c->seg.L;
  HIPCHK(launch_residual(c->dev, L, c->fp32, true, c->u, c->f, c->lam, c->b, c->bxf, c->r, c->part, nullptr, st));
  HIPCHK(launch_cg_init(c->dev, L, c->part, c->opts.inner_tol, c->opts.inner_abs, c->scal, c->ndone, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->opts.timing) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
  }
  const int n_sub = (int)c->subs.size();
  int launches = 0;
  for (int t = 0; t <= c->opts.max_inner; ++t) {
    void* pold = (t & 1) ? c->p1 : c->p0;
    void* pnew = (t & 1) ? c->p0 : c->p1;
    HIPCHK(launch_cg_apply(c->dev, L, c->fp32, t, c->opts.max_inner, c->r, pold, pnew, c->q, c->part, c->scal,
                           c->ndone, c->counters, c->flags, st));
    ++launches;
    if (t == c->opts.max_inner) break;
    HIPCHK(launch_cg_update(c->dev, L, c->fp32, t, c->x, pnew, c->r, c->q, c->part, c->scal, c->ndone, c->flags,
                            st));
    ++launches;
    if ((t & 7) == 7) {
      HIPCHK(hipMemcpyAsync(c->h_ndone, c->ndone, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (*c->h_ndone >= n_sub) break;
    }
  }
  if (c->opts.timing) {
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    c->kernel_ms += ms;
    c->kernel_launches += launches;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  HIPCHK(launch_add_correction(c->dev, L, c->fp32, c->u, c->x, c->scal, st));
  HIPCHK(launch_exchange(c->d_expairs, (int32_t)c->pairs.size(), c->max_face_na, c->max_face_nb, c->u, c->lam, c->f,
                         c->b, c->fxf, c->bxf, st));
  return SOS_OK;
}

int build_graph(sos_ctx* c, int k) {
  invalidate_graph(c);
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = SOS_OK;
  for (int i = 0; i < k && rc == SOS_OK; ++i)
    rc = enqueue_batched_iteration(c, nullptr, nullptr);
  if (rc == SOS_OK) rc = enqueue_check(c, nullptr);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc != SOS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(SOS_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  c->graph = g;
  HIPCHK(hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
  c->graph_k = k;
  return SOS_OK;
}

// Text of a BreakBits word.
std::string break_text(int32_t bits) {
  std::string t;
  auto add = [&](int32_t b, const char* w) {
    if (bits & b) t += (t.empty() ? "" : ", ") + std::string(w);
  };
  add(kBrkCurvature, "non-positive curvature p'Ap in a subdomain CG");
  add(kBrkNonFinite, "non-finite value in a subdomain CG");
  add(kBrkBarrier, "a team member gave up waiting at the team barrier");
  add(kBrkLaunch, "launch shape does not fit the fused kernel variant");
  return t;
}

// SOS_LOG=1 in the environment: one line per convergence check on stderr.
bool log_checks() {
  const char* v = getenv("SOS_LOG");
  return v && *v && strcmp(v, "0") != 0;
}

void history_reset(sos_ctx* c) {
  c->hist_outer.clear();
  c->hist_res.clear();
  c->outer_total = 0;
}

// The fused kernel scales the previous direction vectors by beta = 0 in its
// first CG iteration instead of selecting zero, so they must hold finite
// values: cleared before every run of outer iterations and before tuning
// (fresh allocations, or a run that broke down, may hold anything); every
// launch that does not break down leaves them finite. Outside any graph.
int zero_directions(sos_ctx* c) {
  const size_t bytes = (size_t)c->n_local * (c->fp32 ? sizeof(float) : sizeof(double));
  for (void* v : {c->p0, c->p1, c->s0, c->s1}) HIPCHK(hipMemsetAsync(v, 0, bytes, c->stream));
  return SOS_OK;
}

// Runs outer iterations until the residual <= tol (tol <= 0: exactly max_outer
// iterations with one check every check_every). Every check reads the global
// residual and the solve's breakdown bits (one mapped host word each); a set
// bit ends the run with SOS_EBREAKDOWN. Fills stats.
int run_outer(sos_ctx* c, double tol, int max_outer, sos_stats* stats, bool* converged) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = c->stream;
  *c->h_counters = 0;
  // cleared outside any graph (a captured memset node is avoided on purpose)
  HIPCHK(hipMemsetAsync(c->counters, 0, 2 * sizeof(unsigned long long), st));
  HIPCHK(hipMemsetAsync(c->flags, 0, sizeof(int32_t), st));
  if (c->opts.mode == SOS_BATCHED) {
    int rc = zero_directions(c);
    if (rc) return rc;
  }
  // lambda may have changed since the last exchange (state set, new load)
  HIPCHK(launch_shell_rhs(c->dev, c->seg.L, c->f, c->lam, c->b, c->fxf, c->bxf, st));
  c->h_res[1] = 0.0;
  c->kernel_ms = 0.0;
  c->kernel_launches = 0;
  const bool batched = c->opts.mode == SOS_BATCHED;
  const bool log = log_checks();
  if (batched) {
    int rc = ensure_fmap(c);
    if (rc) return rc;
  }
  // HIP events recorded inside a graph cannot be read back with
  // hipEventElapsedTime: timed runs launch eagerly; so do cooperative team
  // launches (not captured)
  bool plain = c->fused_team == 1;
  if (batched && !plain &&
      launch_fused_cg(c->dev, c->seg.L, c->fp32, c->fused_threads, c->fused_cpt, c->fused_lds, fused_args(c),
                      c->stream, &plain) != hipSuccess)
    plain = false;
  const bool graph = batched && c->opts.use_graph && !c->opts.timing && plain;
  const int every = c->opts.check_every;
  int done = 0, checks = 0;
  int32_t brk = 0;
  double res = INFINITY, best = INFINITY;
  int best_at = 0;
  *converged = false;
  std::vector<hipEvent_t> evs;
  char range[96];
  while (done < max_outer) {
    int k = std::min(every, max_outer - done);
    snprintf(range, sizeof range, "sos outer %d-%d", c->outer_total + 1, c->outer_total + k);
    roctxRangePushA(range);
    if (graph) {
      if (c->graph_k != k) {
        int rc = build_graph(c, k);
        if (rc) {
          roctxRangePop();
          return rc;
        }
      }
      HIPCHK(hipGraphLaunch(c->gexec, st));
    } else {
      for (int i = 0; i < k; ++i) {
        if (batched) {
          hipEvent_t e0 = nullptr, e1 = nullptr;
          if (c->opts.timing) {
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            evs.push_back(e0);
            evs.push_back(e1);
          }
          int rc = enqueue_batched_iteration(c, e0, e1);
          if (rc) return rc;
        } else {
          int rc = stepwise_iteration(c);
          if (rc) return rc;
        }
      }
      int rc = enqueue_check(c, nullptr);
      if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(st));
    roctxRangePop();
    if (c->opts.timing) {
      std::vector<hipEvent_t>& E = evs;
      for (size_t i = 0; i + 1 < E.size(); i += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, E[i], E[i + 1]));
        c->kernel_ms += ms;
        c->kernel_launches += 1;
      }
      for (auto e : evs) (void)hipEventDestroy(e);
      evs.clear();
    }
    done += k;
    c->outer_total += k;
    ++checks;
    res = c->h_res[0];
    brk = (int32_t)c->h_res[1];
    c->hist_outer.push_back(c->outer_total);
    c->hist_res.push_back(res);
    if (log) fprintf(stderr, "sos: outer %d residual %.6e%s\n", c->outer_total, res, brk ? " (breakdown)" : "");
    if (brk || !std::isfinite(res)) break;
    if (tol > 0.0 && res <= tol) {
      *converged = true;
      break;
    }
    // stagnation: no 1% improvement of the best residual for kStallOuter
    // outer iterations (e.g. an outer target below the inner solves' floor)
    if (res < 0.99 * best) {
      best = res;
      best_at = done;
    } else if (tol > 0.0 && done - best_at >= kStallOuter) {
      break;
    }
  }
  HIPCHK(hipMemcpyAsync(c->h_counters, c->counters, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  if (stats) {
    stats->outer_iters = done;
    stats->checks = checks;
    stats->inner_iters = (int64_t)c->h_counters[0];
    stats->rel_residual = res;
    stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    stats->kernel_ms = c->kernel_ms;
    stats->kernel_launches = c->kernel_launches;
    stats->kernel_bytes = (double)c->h_counters[1];
    stats->block = c->fused_threads;
    stats->cols_per_thread = c->fused_cpt;
    stats->wave_rows = c->fused_ra;
    stats->resident = fused_args(c).res;
    stats->team = c->fused_team;
  }
  if (brk)
    return fail(SOS_EBREAKDOWN, "inner solve breakdown after %d outer iterations: %s", c->outer_total,
                break_text(brk).c_str());
  if (!std::isfinite(res)) return fail(SOS_EBREAKDOWN, "non-finite global residual");
  return SOS_OK;
}

int write_phi(sos_ctx* c, double* phi) {
  HIPCHK(launch_fill(phi, c->n_nodes, 0.0, c->stream));
  int rc = enqueue_check(c, phi);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  return SOS_OK;
}

int reset_state(sos_ctx* c) {
  HIPCHK(launch_fill(c->u, c->n_local, 0.0, c->stream));
  HIPCHK(launch_fill(c->lam, c->n_lam, 0.0, c->stream));
  return SOS_OK;
}

// A candidate replaces the tuner's best only when it is faster by more than
// the launch-to-launch noise (1 %): the earliest of near-equal shapes wins, so
// repeated tunings of one problem agree.
constexpr double kTuneMargin = 0.99;

// Autotuner: time every candidate block shape of the fused kernel with every
// uniform team size on the first inner solve of the current load (u = 0,
// lambda = 0), keep the fastest; then, for subdomains of uneven size (more
// than one size bucket), search each bucket's team size in turn (smallest
// bucket first, two passes) with the others fixed. The result is cached per (arch,
// subdomain geometry, precision, inner tolerance).
int autotune(sos_ctx* c) {
  if (c->tuned) return SOS_OK;
  c->tuned = true;
  const std::string key = tune_key(c);
  // a block shape or team size fixed by the caller is kept: such a partial
  // search neither reads nor writes the cache (its entries hold full searches)
  const bool partial = c->opts.block != 0 || c->opts.team != 0;
  int th = 0, cp = 0, ra = 0, res = 0;
  std::vector<int32_t> bt;
  if (!partial && tune_lookup(key, &th, &cp, &bt, &ra, &res) && (int)bt.size() == c->n_buckets &&
      fused_shape(c, th, cp, ra, res && c->opts.resident) == SOS_OK && set_bucket_teams(c, bt) == SOS_OK)
    return SOS_OK;
  // block shapes are tuned unless fixed by opts.block, team sizes unless fixed by opts.team
  std::vector<Shape> shapes;
  if (c->opts.block) shapes.push_back({c->fused_threads, c->fused_cpt, c->fused_ra, c->fused_res});
  else shapes = fused_candidates(c);
  auto team_ok = [&](int t, int bucket) {  // every subdomain of the bucket (-1: all) has 2t planes
    for (size_t i = 0; i < c->subs.size(); ++i)
      if ((bucket < 0 || c->sub_bucket[i] == bucket) && c->subs[i].n[2] < 2 * t) return false;
    return true;
  };
  std::vector<int> teams;
  if (c->opts.team) teams.push_back(c->opts.team);
  else
    for (int t : {1, 2, 4, 8})
      if (team_ok(t, -1)) teams.push_back(t);
  hipStream_t st = c->stream;
  if (int rc0 = zero_directions(c)) return rc0;
  // the trial launches solve the first outer iteration's problem: the
  // right-hand side on the boundary shell as a run starts it
  HIPCHK(launch_shell_rhs(c->dev, c->seg.L, c->f, c->lam, c->b, c->fxf, c->bxf, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // fastest of three launches of the current shape and teams (INFINITY: unusable)
  auto time_config = [&](double* out) -> int {
    *out = INFINITY;
    int rc = ensure_fmap(c);
    if (rc) return rc;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(launch_fill(c->u, c->n_local, 0.0, st));
      HIPCHK(launch_residual(c->dev, c->seg.L, c->fp32, false, c->u, c->f, c->lam, c->b, c->bxf, c->r, c->part,
                             c->fused_team > 1 ? c->team_part : nullptr, st));
      HIPCHK(hipEventRecord(e0, st));
      if (launch_fused_cg(c->dev, c->seg.L, c->fp32, c->fused_threads, c->fused_cpt, c->fused_lds, fused_args(c),
                          st) != hipSuccess) {
        (void)hipGetLastError();  // e.g. a team grid that cannot be co-resident
        *out = INFINITY;
        return SOS_OK;
      }
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      *out = std::min(*out, (double)ms);
    }
    return SOS_OK;
  };
  double best = INFINITY;
  Shape bs{c->fused_threads, c->fused_cpt, c->fused_ra, c->fused_res};
  std::vector<int32_t> bteams(c->n_buckets, c->fused_team);
  int rc = SOS_OK;
  for (int team : teams)
    for (auto& cd : shapes) {
      if (fused_shape(c, cd.threads, cd.cpt, cd.ra, cd.res) != SOS_OK || set_team(c, team) != SOS_OK) continue;
      if (cd.res && !fused_args(c).res) continue;  // p and x do not fit in LDS with this team
      double ms = INFINITY;
      if ((rc = time_config(&ms))) break;
      if (ms < best * kTuneMargin) {
        best = ms;
        bs = cd;
        bteams.assign(c->n_buckets, team);
      }
    }
  // per-bucket team sizes with the best shape: two passes of coordinate
  // descent, smallest bucket first (shrinking the small subdomains' teams
  // frees co-resident blocks that the large ones' teams then need)
  if (!rc && c->n_buckets > 1 && !c->opts.team && std::isfinite(best) &&
      fused_shape(c, bs.threads, bs.cpt, bs.ra, bs.res) == SOS_OK) {
    for (int pass = 0; pass < 2 * c->n_buckets && !rc; ++pass) {
      const int b = c->n_buckets - 1 - pass % c->n_buckets;
      for (int t : {1, 2, 4, 8}) {
        if (t == bteams[b] || !team_ok(t, b)) continue;
        std::vector<int32_t> trial = bteams;
        trial[b] = t;
        if (set_bucket_teams(c, trial) != SOS_OK) continue;
        if (bs.res && !fused_args(c).res) continue;
        double ms = INFINITY;
        if ((rc = time_config(&ms))) break;
        if (ms < best * kTuneMargin) {
          best = ms;
          bteams = trial;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  HIPCHK(launch_fill(c->u, c->n_local, 0.0, st));
  HIPCHK(hipStreamSynchronize(st));
  rc = fused_shape(c, bs.threads, bs.cpt, bs.ra, bs.res);
  if (!rc) rc = set_bucket_teams(c, bteams);
  if (rc) return rc;
  c->tune_ms = best;
  invalidate_graph(c);
  if (!partial) tune_store(key, bs.threads, bs.cpt, bteams, bs.ra, bs.res, best);
  return SOS_OK;
}

int solve_common(sos_ctx* c, double tol, double* phi, sos_stats* stats) {
  if (!(tol > 0.0)) return fail(SOS_EINVAL, "tol must be > 0");
  if (!phi) return fail(SOS_EINVAL, "phi_nodes is NULL");
  int rc = reset_state(c);
  if (rc) return rc;
  if (c->opts.mode == SOS_BATCHED && (rc = autotune(c))) return rc;
  history_reset(c);
  bool conv = false;
  rc = run_outer(c, tol, c->opts.max_outer, stats, &conv);
  if (rc) return rc;
  rc = write_phi(c, phi);
  if (rc) return rc;
  if (!conv)
    return fail(SOS_ENOCONV, "no convergence to %g after %d outer iterations (residual %g%s)", tol,
                stats ? stats->outer_iters : c->opts.max_outer, *c->h_res,
                (stats && stats->outer_iters < c->opts.max_outer) ? ", stagnated" : "");
  return SOS_OK;
}

}  // namespace

// ============================================================================ C-ABI

extern "C" {

const char* sos_last_error(void) { return g_err.c_str(); }

int sos_opts_default(sos_opts* o, int32_t precision) {
  if (!o) return fail(SOS_EINVAL, "opts is NULL");
  std::memset(o, 0, sizeof *o);
  o->precision = precision;
  o->mode = precision == SOS_FP32_INNER ? SOS_BATCHED : SOS_STEPWISE;
  o->max_outer = 100000;
  o->max_inner = 500;
  o->check_every = 1;
  o->use_graph = 1;
  o->inner_tol = precision == SOS_FP32_INNER ? 1e-2 : 0.0;
  o->inner_abs = precision == SOS_FP32_INNER ? 0.0 : 1e-10;
  o->G = 6.672e-11;
  o->stream = nullptr;
  o->block = 0;
  o->timing = 0;
  o->wave_rows = 0;
  o->resident = 1;
  o->schedule = 1;
  return SOS_OK;
}

int sos_setup(const sos_mesh* mesh, const sos_partition* part, const sos_robin* robin, const sos_opts* opts,
              sos_ctx** out) {
  return sos_setup_batch(mesh, part, 1, robin, opts, out);
}

int sos_setup_batch(const sos_mesh* mesh, const sos_partition* part, int32_t copies, const sos_robin* robin,
                    const sos_opts* opts, sos_ctx** out) {
  if (!out) return fail(SOS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mesh || !part || !robin || !opts) return fail(SOS_EINVAL, "NULL argument");
  if (copies < 1 || copies > kMaxCopies) return fail(SOS_EINVAL, "copies must be in [1, %d]", kMaxCopies);
  int rc = check_opts(opts);
  if (rc) return rc;
  bool any_dir = false;
  for (int a = 0; a < 3; ++a) {
    if (mesh->ne[a] < 1) return fail(SOS_EINVAL, "mesh.ne[%d] must be >= 1", a);
    if (!(mesh->len[a] > 0.0) || !std::isfinite(mesh->len[a])) return fail(SOS_EINVAL, "mesh.len[%d] must be > 0", a);
  }
  for (int f = 0; f < 6; ++f) {
    if (mesh->bc[f] != SOS_DIRICHLET && mesh->bc[f] != SOS_NEUMANN) return fail(SOS_EINVAL, "mesh.bc[%d] invalid", f);
    any_dir |= mesh->bc[f] == SOS_DIRICHLET;
  }
  if (!any_dir) return fail(SOS_EINVAL, "at least one outer face must be Dirichlet (pure Neumann is singular)");
  std::vector<int32_t> bounds[3];
  for (int a = 0; a < 3; ++a) {
    const int np = part->nparts[a], ne = mesh->ne[a];
    if (np < 1 || np > ne) return fail(SOS_EINVAL, "partition.nparts[%d] must be in [1, ne]", a);
    bounds[a].push_back(0);
    if (part->cuts[a]) {
      for (int k = 0; k < np - 1; ++k) {
        int v = part->cuts[a][k];
        if (v <= bounds[a].back() || v >= ne) return fail(SOS_EINVAL, "partition.cuts[%d] must increase strictly inside (0, ne)", a);
        bounds[a].push_back(v);
      }
    } else {
      if (ne % np) return fail(SOS_EINVAL, "equal split: nparts[%d] must divide ne[%d]", a, a);
      for (int k = 1; k < np; ++k) bounds[a].push_back(k * (ne / np));
    }
    bounds[a].push_back(ne);
  }
  sos_ctx* c = new (std::nothrow) sos_ctx();
  if (!c) return fail(SOS_ENOMEM, "host allocation failed");
  c->mesh = *mesh;
  c->opts = *opts;
  c->fp32 = opts->precision == SOS_FP32_INNER;
  Geom& g = c->geo;
  for (int a = 0; a < 3; ++a) {
    g.ne[a] = mesh->ne[a];
    g.nn[a] = 2 * mesh->ne[a] + 1;
    g.h[a] = mesh->len[a] / mesh->ne[a];
    g.ks[a] = 1.0 / (3.0 * g.h[a]);
    g.ms[a] = g.h[a] / 30.0;
    g.nparts[a] = part->nparts[a];
  }
  for (int f = 0; f < 6; ++f) g.bc[f] = mesh->bc[f];
  g.n_sub = part->nparts[0] * part->nparts[1] * part->nparts[2];
  c->n_nodes = (int64_t)g.nn[0] * g.nn[1] * g.nn[2];
  // subdomains
  const int Px = g.nparts[0], Py = g.nparts[1], Pz = g.nparts[2];
  int64_t off = 0;
  c->subs.resize(g.n_sub);
  for (int pz = 0; pz < Pz; ++pz)
    for (int py = 0; py < Py; ++py)
      for (int px = 0; px < Px; ++px) {
        const int s = px + Px * (py + Py * pz);
        SubDesc& d = c->subs[s];
        const int pp[3] = {px, py, pz};
        int64_t n = 1;
        for (int a = 0; a < 3; ++a) {
          const int e0 = bounds[a][pp[a]], e1 = bounds[a][pp[a] + 1];
          int klo = 0, khi = 2 * (e1 - e0);
          if (e0 == 0 && mesh->bc[2 * a] == SOS_DIRICHLET) klo = 1;
          if (e1 == mesh->ne[a] && mesh->bc[2 * a + 1] == SOS_DIRICHLET) khi -= 1;
          d.n[a] = khi - klo + 1;
          d.klo[a] = klo;
          d.ne2[a] = 2 * (e1 - e0);
          d.lo[a] = 2 * e0 + klo;
          d.pidx[a] = pp[a];
          d.e0[a] = e0;
          d.elo[a] = d.ehi[a] = 0.0;
          d.qlo[a] = d.qhi[a] = 0.0;
          n *= d.n[a];
        }
        for (int k = 0; k < 6; ++k) d.face[k] = -1;
        d.off = off;
        off = align64(off + n);
        c->max_n = std::max<int>(c->max_n, (int)n);
      }
  c->n_local = off;
  // directed faces: by s, axis, side
  int64_t loff = 0;
  for (int s = 0; s < g.n_sub; ++s) {
    SubDesc& d = c->subs[s];
    for (int a = 0; a < 3; ++a)
      for (int side = 0; side < 2; ++side) {
        int q[3] = {d.pidx[0], d.pidx[1], d.pidx[2]};
        q[a] += side ? 1 : -1;
        if (q[a] < 0 || q[a] >= g.nparts[a]) continue;
        FaceDesc F{};
        F.s = s;
        F.j = q[0] + Px * (q[1] + Py * q[2]);
        F.axis = a;
        F.side = side;
        const int ta = a == 0 ? 1 : 0, tb = a == 2 ? 1 : 2;
        F.na = d.n[ta];
        F.nb = d.n[tb];
        F.lam_off = loff;
        F.opp = -1;
        loff += (int64_t)F.na * F.nb;
        c->max_face = std::max(c->max_face, F.na * F.nb);
        c->max_face_na = std::max(c->max_face_na, F.na);
        c->max_face_nb = std::max(c->max_face_nb, F.nb);
        d.face[2 * a + side] = (int32_t)c->faces.size();
        c->faces.push_back(F);
      }
  }
  c->n_lam = loff;
  for (auto& F : c->faces) {
    const SubDesc& dj = c->subs[F.j];
    F.opp = dj.face[2 * F.axis + (1 - F.side)];
    if (F.s < F.j) c->pairs.push_back((int32_t)(&F - &c->faces[0]));
  }
  choose_axes(c, opts->march);
  // independent copies of the problem: subdomains, faces and vectors repeat
  // copy after copy (copy c's subdomain s is c * n_sub + s)
  {
    const int ns = g.n_sub, nf = (int)c->faces.size(), np = (int)c->pairs.size();
    const int64_t nl = c->n_local, nlam = c->n_lam;
    if ((int64_t)ns * copies > INT32_MAX / 2 || (int64_t)nf * copies > INT32_MAX / 2) {
      release(c);
      return fail(SOS_EINVAL, "too many subdomains in %d copies", copies);
    }
    for (auto& d : c->subs) d.copy = d.sbase = 0;
    c->subs.resize((size_t)ns * copies);
    c->faces.resize((size_t)nf * copies);
    for (int cc = 1; cc < copies; ++cc) {
      for (int s = 0; s < ns; ++s) {
        SubDesc d = c->subs[s];
        d.off += cc * nl;
        d.copy = cc;
        d.sbase = cc * ns;
        for (int f = 0; f < 6; ++f)
          if (d.face[f] >= 0) d.face[f] += cc * nf;
        c->subs[(size_t)cc * ns + s] = d;
      }
      for (int f = 0; f < nf; ++f) {
        FaceDesc F = c->faces[f];
        F.s += cc * ns;
        F.j += cc * ns;
        F.opp += cc * nf;
        F.lam_off += cc * nlam;
        c->faces[(size_t)cc * nf + f] = F;
      }
      for (int p = 0; p < np; ++p) c->pairs.push_back(c->pairs[p] + cc * nf);
    }
    c->n_local = nl * copies;
    c->n_lam = nlam * copies;
    c->n_nodes *= copies;
    g.n_sub = ns * copies;
    g.copies = copies;
  }
  // x-boundary right-hand sides (local axis order): 2 n1 n2 values each
  for (auto& d : c->subs) {
    d.xoff = c->n_xface;
    c->n_xface += 2 * (int64_t)d.n[1] * d.n[2];
  }
  rc = apply_robin(c, robin);
  if (rc) {
    release(c);
    return rc;
  }
  // device and launch limits
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    release(c);
    return fail(SOS_ESTATE, "no usable HIP device");
  }
  c->lds_limit = prop.sharedMemPerBlock;
  if ((rc = scratch_address(&c->scratch))) {
    release(c);
    return rc;
  }
  {
    const size_t ex_lds =
        2 * sizeof(double) * (size_t)(c->max_face_na + 4) * (size_t)(exchange_rows(c->max_face_na) + 4);
    if (ex_lds > c->lds_limit) {
      release(c);
      return fail(SOS_EINVAL, "interface face of %d nodes along its first axis needs %zu bytes of LDS (limit %zu)",
                  c->max_face_na, ex_lds, (size_t)prop.sharedMemPerBlock);
    }
  }
  c->tuned = opts->block != 0 && opts->team != 0;
  if ((rc = build_seg(c)) || (rc = fused_shape(c, opts->block, 0, opts->wave_rows, opts->resident)) || (rc = set_team(c, opts->team ? opts->team : 1))) {
    release(c);
    return rc;
  }
  // fused order: largest first; block table capacity: sum of teams (at most
  // kMaxTeam per subdomain) plus the padding of eight queues
  make_buckets(c);
  c->fmap_cap = (size_t)kMaxTeam * g.n_sub + 8 * kMaxTeam;
  c->order.resize(g.n_sub);
  for (int s = 0; s < g.n_sub; ++s) c->order[s] = s;
  std::stable_sort(c->order.begin(), c->order.end(), [&](int a, int b) {
    const SubDesc &A = c->subs[a], &B = c->subs[b];
    return (int64_t)A.n[0] * A.n[1] * A.n[2] > (int64_t)B.n[0] * B.n[1] * B.n[2];
  });
  // allocations
  const size_t es = c->fp32 ? 4 : 8;
  Dev tmp{nullptr, nullptr, g, 0, 0};
  for (const SubDesc& d : c->subs) c->max_shell = std::max(c->max_shell, shell_nodes(d.n[0], d.n[1], d.n[2]));
  c->n_norm_blocks = c->seg.L.nblocks + shell_blocks(tmp, c->max_shell);
  if ((rc = dalloc(&c->d_subs, c->subs.size())) || (rc = dalloc(&c->d_faces, c->faces.size())) ||
      (rc = dalloc(&c->d_expairs, c->pairs.size())) || (rc = dalloc(&c->d_fmap, c->fmap_cap)) ||
      (rc = dalloc(&c->seg.d_blocks, c->seg.blocks.size())) || (rc = dalloc(&c->seg.d_bfirst, c->seg.bfirst.size())) ||
      (rc = dalloc(&c->u, c->n_local)) || (rc = dalloc(&c->f, c->n_local)) || (rc = dalloc(&c->lam, c->n_lam)) ||
      (rc = dalloc(&c->b, c->n_local)) || (rc = dalloc(&c->fxf, c->n_xface)) ||
      (rc = dalloc(&c->bxf, c->n_xface)) ||
      (rc = dalloc(&c->ut, c->n_local)) || (rc = dalloc(&c->rho, c->n_local)) ||
      (rc = dalloc_v(&c->r, c->n_local * es)) || (rc = dalloc_v(&c->x, c->n_local * es)) ||
      (rc = dalloc_v(&c->p0, c->n_local * es)) || (rc = dalloc_v(&c->p1, c->n_local * es)) ||
      (rc = dalloc_v(&c->q, c->n_local * es)) || (rc = dalloc_v(&c->r1, c->n_local * es)) ||
      (rc = dalloc_v(&c->w1, c->n_local * es)) || (rc = dalloc_v(&c->s0, c->n_local * es)) ||
      (rc = dalloc_v(&c->s1, c->n_local * es)) || (rc = dalloc(&c->part, 3 * c->seg.blocks.size())) ||
      (rc = dalloc(&c->part_norm, 2 * (size_t)c->n_norm_blocks)) || (rc = dalloc(&c->d_res, 4 + (size_t)copies)) ||
      (rc = dalloc(&c->scal, c->subs.size())) || (rc = dalloc(&c->ndone, 1)) || (rc = dalloc(&c->counters, 2)) ||
      (rc = dalloc(&c->flags, 1)) ||
      (rc = dalloc(&c->team_part, c->subs.size() * kMaxTeam * 2 * 4))) {
    release(c);
    return rc;
  }
  if (hipHostMalloc((void**)&c->h_res, 2 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&c->d_hres, c->h_res, 0) != hipSuccess ||
      hipHostMalloc((void**)&c->h_ndone, sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_counters, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
    release(c);
    return fail(SOS_ENOMEM, "hipHostMalloc failed");
  }
  c->h_res[0] = INFINITY;
  c->h_res[1] = 0.0;
  if (opts->stream) {
    c->stream = (hipStream_t)opts->stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      release(c);
      return fail(SOS_EHIP, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  c->seg.L.blocks = c->seg.d_blocks;
  c->seg.L.bfirst = c->seg.d_bfirst;
  c->dev.subs = c->d_subs;
  c->dev.faces = c->d_faces;
  c->dev.geo = g;
  c->dev.n_faces = (int32_t)c->faces.size();
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(c->d_subs, c->subs.data(), c->subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess && !c->faces.empty())
    e = hipMemcpy(c->d_faces, c->faces.data(), c->faces.size() * sizeof(FaceDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = upload_expairs(c);
  if (e == hipSuccess)
    e = hipMemcpy(c->seg.d_blocks, c->seg.blocks.data(), c->seg.blocks.size() * sizeof(BlockDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->seg.d_bfirst, c->seg.bfirst.data(), c->seg.bfirst.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->f, 0, c->n_local * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->b, 0, c->n_local * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->fxf, 0, c->n_xface * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->bxf, 0, c->n_xface * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->u, 0, c->n_local * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->lam, 0, std::max<int64_t>(1, c->n_lam) * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->rho, 0, c->n_local * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->flags, 0, sizeof(int32_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release(c);
    return fail(SOS_EHIP, "setup copies: %s", hipGetErrorString(e));
  }
  *out = c;
  return SOS_OK;
}

int sos_set_robin(sos_ctx* c, const sos_robin* robin) {
  if (!c) return fail(SOS_EINVAL, "ctx is NULL");
  int rc = apply_robin(c, robin);
  if (rc) return rc;
  invalidate_graph(c);
  hipError_t e = hipMemcpy(c->d_subs, c->subs.data(), c->subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess && !c->faces.empty())
    e = hipMemcpy(c->d_faces, c->faces.data(), c->faces.size() * sizeof(FaceDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = upload_expairs(c);
  if (e != hipSuccess) return fail(SOS_EHIP, "set_robin copies: %s", hipGetErrorString(e));
  return SOS_OK;
}

int sos_set_opts(sos_ctx* c, const sos_opts* o) {
  if (!c || !o) return fail(SOS_EINVAL, "NULL argument");
  int rc = check_opts(o);
  if (rc) return rc;
  if ((o->precision == SOS_FP32_INNER) != (c->fp32 != 0)) return fail(SOS_EINVAL, "precision is fixed at setup");
  if (o->stream && o->stream != c->stream) return fail(SOS_EINVAL, "the stream is fixed at setup");
  if (o->march != c->opts.march) return fail(SOS_EINVAL, "the march axes are fixed at setup");
  const int old_block = c->opts.block, old_team = c->opts.team, old_rows = c->opts.wave_rows,
            old_res = c->opts.resident, old_sched = c->opts.schedule;
  const double old_tol = c->opts.inner_tol, old_abs = c->opts.inner_abs;
  void* st = c->opts.stream;
  c->opts = *o;
  c->opts.stream = st;
  const bool retune = o->block != old_block || o->team != old_team || o->wave_rows != old_rows ||
                      o->resident != old_res || o->inner_tol != old_tol || o->inner_abs != old_abs;
  if (retune) {
    rc = fused_shape(c, o->block, 0, o->wave_rows, o->resident);
    if (!rc) rc = set_team(c, o->team ? o->team : 1);
    if (rc) return rc;
    c->tuned = o->block != 0 && o->team != 0;
  }
  if (o->schedule != old_sched) c->fmap_dirty = true;  // back to the fixed order
  invalidate_graph(c);
  return SOS_OK;
}

int sos_axes(const sos_ctx* c, int32_t* perm) {
  if (!c || !perm) return fail(SOS_EINVAL, "NULL argument");
  for (size_t i = 0; i < c->subs.size(); ++i)
    for (int a = 0; a < 3; ++a) perm[3 * i + a] = c->subs[i].perm[a];
  return SOS_OK;
}

int sos_teams(const sos_ctx* c, int32_t* teams) {
  if (!c || !teams) return fail(SOS_EINVAL, "NULL argument");
  for (size_t i = 0; i < c->sub_team.size(); ++i) teams[i] = c->sub_team[i];
  return SOS_OK;
}

int sos_set_teams(sos_ctx* c, const int32_t* teams) {
  if (!c || !teams) return fail(SOS_EINVAL, "NULL argument");
  int rc = set_teams(c, std::vector<int32_t>(teams, teams + c->subs.size()));
  if (rc) return rc;
  c->tuned = true;  // keep these teams and the current block shape
  return SOS_OK;
}

int sos_faces(const sos_ctx* c, int32_t* n, int32_t* sjas) {
  if (!c || !n) return fail(SOS_EINVAL, "NULL argument");
  *n = (int32_t)c->faces.size();
  if (sjas)
    for (size_t f = 0; f < c->faces.size(); ++f) {
      sjas[4 * f] = c->faces[f].s;
      sjas[4 * f + 1] = c->faces[f].j;
      sjas[4 * f + 2] = c->faces[f].axis;
      sjas[4 * f + 3] = c->faces[f].side;
    }
  return SOS_OK;
}

int sos_layout(const sos_ctx* c, int32_t* n_sub, int64_t* offsets, int32_t* dims, int32_t* lo, int64_t* face_off) {
  if (!c || !n_sub) return fail(SOS_EINVAL, "NULL argument");
  *n_sub = (int32_t)c->subs.size();
  for (size_t s = 0; s < c->subs.size(); ++s) {
    if (offsets) offsets[s] = c->subs[s].off;
    for (int a = 0; a < 3; ++a) {
      if (dims) dims[3 * s + a] = c->subs[s].n[a];
      if (lo) lo[3 * s + a] = c->subs[s].lo[a];
    }
  }
  if (offsets) offsets[c->subs.size()] = c->n_local;
  if (face_off) {
    for (size_t f = 0; f < c->faces.size(); ++f) face_off[f] = c->faces[f].lam_off;
    face_off[c->faces.size()] = c->n_lam;
  }
  return SOS_OK;
}

int sos_set_density(sos_ctx* c, const double* drho) {
  if (!c || !drho) return fail(SOS_EINVAL, "NULL argument");
  HIPCHK(launch_load_density(c->dev, c->max_n, drho, c->opts.G, c->f, c->stream));
  HIPCHK(copy_load_to_rhs(c));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->have_load = true;
  return SOS_OK;
}

int sos_batch_residuals(sos_ctx* c, double* res) {
  if (!c || !res) return fail(SOS_EINVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(res, c->d_res + 3, (size_t)c->geo.copies * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SOS_OK;
}

int sos_batch_rates(sos_ctx* c, const double* drho, int32_t n_first, int32_t n_second, double* rates,
                    double* res_first, double* res_second, int32_t* best, sos_stats* stats) {
  if (!c || !drho || !rates) return fail(SOS_EINVAL, "NULL argument");
  if (n_first < 1 || n_second <= n_first) return fail(SOS_EINVAL, "need 1 <= n_first < n_second");
  const int B = c->geo.copies;
  HIPCHK(launch_load_density(c->dev, c->max_n, drho, c->opts.G, c->f, c->stream));
  HIPCHK(copy_load_to_rhs(c));
  c->have_load = true;
  int rc = reset_state(c);
  if (rc) return rc;
  if (c->opts.mode == SOS_BATCHED && (rc = autotune(c))) return rc;
  history_reset(c);
  bool conv = false;
  std::vector<double> r1(B), r2(B);
  sos_stats s1{}, s2{};
  if ((rc = run_outer(c, 0.0, n_first, &s1, &conv)) || (rc = sos_batch_residuals(c, r1.data()))) return rc;
  if ((rc = run_outer(c, 0.0, n_second - n_first, &s2, &conv)) || (rc = sos_batch_residuals(c, r2.data())))
    return rc;
  int arg = -1;
  for (int i = 0; i < B; ++i) {
    // rate per outer iteration between the two checks
    rates[i] = (r1[i] > 0.0 && std::isfinite(r1[i]) && std::isfinite(r2[i]))
                   ? std::pow(r2[i] / r1[i], 1.0 / double(n_second - n_first))
                   : NAN;
    if (res_first) res_first[i] = r1[i];
    if (res_second) res_second[i] = r2[i];
    if (std::isfinite(rates[i]) && (arg < 0 || rates[i] < rates[arg])) arg = i;  // ties: the lower index
  }
  if (best) *best = arg;
  if (stats) {
    *stats = s2;
    stats->outer_iters = s1.outer_iters + s2.outer_iters;
    stats->checks = s1.checks + s2.checks;
    stats->inner_iters = s1.inner_iters + s2.inner_iters;
    stats->seconds = s1.seconds + s2.seconds;
    stats->kernel_ms = s1.kernel_ms + s2.kernel_ms;
    stats->kernel_launches = s1.kernel_launches + s2.kernel_launches;
    stats->kernel_bytes = s1.kernel_bytes + s2.kernel_bytes;
  }
  return arg < 0 ? fail(SOS_EBREAKDOWN, "no copy has a finite rate") : SOS_OK;
}

int sos_solve(sos_ctx* c, const double* drho, double tol, double* phi, sos_stats* stats) {
  if (!c || !drho) return fail(SOS_EINVAL, "NULL argument");
  HIPCHK(launch_load_density(c->dev, c->max_n, drho, c->opts.G, c->f, c->stream));
  HIPCHK(copy_load_to_rhs(c));
  c->have_load = true;
  return solve_common(c, tol, phi, stats);
}

int sos_solve_load(sos_ctx* c, const double* fn, double tol, double* phi, sos_stats* stats) {
  if (!c || !fn) return fail(SOS_EINVAL, "NULL argument");
  if (c->geo.copies > 1) return fail(SOS_EINVAL, "nodal loads are not supported on a context of several copies");
  HIPCHK(launch_load_nodes(c->dev, c->max_n, fn, c->f, c->stream));
  HIPCHK(copy_load_to_rhs(c));
  c->have_load = true;
  return solve_common(c, tol, phi, stats);
}

int sos_adjoint(sos_ctx* c, const double* gphi, double tol, double* grad, double* psi, sos_stats* stats) {
  if (!c || !gphi || !grad) return fail(SOS_EINVAL, "NULL argument");
  if (c->geo.copies > 1) return fail(SOS_EINVAL, "the adjoint is not supported on a context of several copies");
  double* out = psi;
  if (!out) {
    if (!c->psi && dalloc(&c->psi, (size_t)c->n_nodes)) return SOS_ENOMEM;
    out = c->psi;
  }
  HIPCHK(launch_load_nodes(c->dev, c->max_n, gphi, c->f, c->stream));
  HIPCHK(copy_load_to_rhs(c));
  c->have_load = true;
  int rc = solve_common(c, tol, out, stats);
  if (rc != SOS_OK && rc != SOS_ENOCONV) return rc;
  HIPCHK(launch_grad_density(c->geo, out, c->opts.G, grad, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return rc;
}

int sos_iterate(sos_ctx* c, int32_t n, sos_stats* stats) {
  if (!c) return fail(SOS_EINVAL, "ctx is NULL");
  if (n < 1) return fail(SOS_EINVAL, "n must be >= 1");
  if (!c->have_load) return fail(SOS_ESTATE, "no load set (sos_set_density or a solve first)");
  bool conv = false;
  return run_outer(c, 0.0, n, stats, &conv);
}

int sos_residual(sos_ctx* c, double* phi, double* res) {
  if (!c) return fail(SOS_EINVAL, "ctx is NULL");
  int rc = phi ? write_phi(c, phi) : enqueue_check(c, nullptr);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  if (res) *res = c->h_res[0];
  return SOS_OK;
}

int sos_residual_noalloc(sos_ctx* c, double* phi, double* res) {
  if (!c) return fail(SOS_EINVAL, "ctx is NULL");
  if (!c->scratch) return fail(SOS_ESTATE, "no scratch address for this context's device");
  // ut and rho (local layout), the check partials and the result words
  const size_t n_vec = (size_t)align64(c->n_local);
  const size_t n_part = (size_t)align64(2 * (int64_t)c->n_norm_blocks);
  const size_t need = (2 * n_vec + n_part + 4 + (size_t)c->geo.copies) * sizeof(double);
  if (need > kScratchBytes)
    return fail(SOS_EINVAL, "the global residual of %lld local unknowns needs %zu bytes of scratch; the "
                "allocation-free variant holds at most %zu bytes (about %zu local unknowns)",
                (long long)c->n_local, need, kScratchBytes, kScratchBytes / (2 * sizeof(double)) - 8192);
  double* ut = static_cast<double*>(c->scratch);
  double* rho = ut + n_vec;
  double* part = rho + n_vec;
  double* dres = part + n_part;
  hipStream_t st = c->stream;
  if (phi) HIPCHK(launch_fill(phi, c->n_nodes, 0.0, st));
  if (int rc = check_passes(c, ut, rho, part, dres, phi)) return rc;
  HIPCHK(hipStreamSynchronize(st));
  if (res) *res = c->h_res[0];
  return SOS_OK;
}

int sos_get_state(sos_ctx* c, double* u, double* lam) {
  if (!c) return fail(SOS_EINVAL, "ctx is NULL");
  if (u) HIPCHK(hipMemcpyAsync(u, c->u, c->n_local * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (lam && c->n_lam) HIPCHK(hipMemcpyAsync(lam, c->lam, c->n_lam * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SOS_OK;
}

int sos_set_state(sos_ctx* c, const double* u, const double* lam) {
  if (!c) return fail(SOS_EINVAL, "ctx is NULL");
  if (u) HIPCHK(hipMemcpyAsync(c->u, u, c->n_local * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (lam && c->n_lam) HIPCHK(hipMemcpyAsync(c->lam, lam, c->n_lam * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  history_reset(c);
  return SOS_OK;
}

int sos_history(const sos_ctx* c, int32_t cap, int32_t* n, int32_t* outer, double* res) {
  if (!c || !n) return fail(SOS_EINVAL, "NULL argument");
  if (cap < 0) return fail(SOS_EINVAL, "cap must be >= 0");
  *n = (int32_t)c->hist_res.size();
  const size_t m = std::min<size_t>((size_t)cap, c->hist_res.size());
  for (size_t i = 0; i < m; ++i) {
    if (outer) outer[i] = c->hist_outer[i];
    if (res) res[i] = c->hist_res[i];
  }
  return SOS_OK;
}

int sos_inner_iters(sos_ctx* c, int32_t cap, int32_t* n, int32_t* iters) {
  if (!c || !n) return fail(SOS_EINVAL, "NULL argument");
  if (cap < 0) return fail(SOS_EINVAL, "cap must be >= 0");
  *n = (int32_t)c->subs.size();
  const size_t m = std::min<size_t>((size_t)cap, c->subs.size());
  if (m == 0 || !iters) return SOS_OK;
  std::vector<CgScal> h(m);
  HIPCHK(hipMemcpyAsync(h.data(), c->scal, m * sizeof(CgScal), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < m; ++i) iters[i] = h[i].iters;
  return SOS_OK;
}

int sos_debug_barrier(sos_ctx* c, int64_t spin_ticks, int32_t tag_skew) {
  if (!c) return fail(SOS_EINVAL, "ctx is NULL");
  if (spin_ticks < 0) return fail(SOS_EINVAL, "spin_ticks must be >= 0");
  if (tag_skew != 0 && tag_skew != 1) return fail(SOS_EINVAL, "tag_skew must be 0 or 1");
  c->spin_ticks = spin_ticks ? (uint64_t)spin_ticks : (1ull << 27);
  c->tag_skew = tag_skew;
  invalidate_graph(c);
  return SOS_OK;
}

int sos_apply_local(sos_ctx* c, int32_t precision, const void* x, void* y) {
  if (!c || !x || !y) return fail(SOS_EINVAL, "NULL argument");
  if (precision != SOS_FP64 && precision != SOS_FP32_INNER) return fail(SOS_EINVAL, "precision invalid");
  SegLaunch L = c->seg.L;
  if (precision == SOS_FP32_INNER && L.lds32 > c->lds_limit) return fail(SOS_EINVAL, "LDS limit");
  HIPCHK(launch_apply(c->dev, L, precision == SOS_FP32_INNER, x, y, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SOS_OK;
}

void sos_destroy(sos_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  release(c);
}

}  // extern "C"
