// HIP kernels of the Robin-Schwarz subdomain solves (gfx950, wave64): the
// outer-iteration kernels (exchange, glue, global residual, loads) and the
// launchers. The kernel templates live in sos_device.h; the fused CG kernel's
// launches are compiled per columns-per-thread value in sos_fused.hip.
#include "sos_device.h"

namespace sos {

int launch_bound(int cpt) { return cpt == 2 ? 704 : (cpt == 3 ? 512 : 1024); }

// ---------------------------------------------------------------------------- stepwise CG

__global__ void k_cg_init(int n_sub, const int32_t* __restrict__ bfirst, const double* __restrict__ part,
                          double tol_rel, double tol_abs, CgScal* __restrict__ scal, int32_t* ndone) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) *ndone = 0;
  if (s >= n_sub) return;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for (int b = bfirst[s]; b < bfirst[s + 1]; ++b) {
    rz += part[3 * b];
    rr += part[3 * b + 1];
    bb += part[3 * b + 2];
  }
  CgScal c;
  c.rz[0] = rz;
  c.rz[1] = rz;
  c.rr0 = rr;
  c.stop2 = fmax(tol_rel * tol_rel * rr, tol_abs * tol_abs * bb);
  c.done = 0;
  c.iters = 0;
  c.breakdown = 0;
  c.pad = 0;
  scal[s] = c;
}

// ---------------------------------------------------------------------------- block order

// Block table of the fused kernel with one block per subdomain: subdomains in
// decreasing order of the work of their last inner solve, (iterations + 1) x
// nodes, quantised to kOrderBins bins of equal width (equal bins in index
// order). Blocks are dispatched in index order onto compute units as these free
// up, so when the grid takes several rounds of resident blocks this is list
// scheduling with the longest jobs first. One workgroup of NT threads (sm:
// order_lds_bytes(NT) bytes of LDS); a counting sort whose ranks inside a
// chunk come from wave ballots.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 64;
constexpr size_t order_lds_bytes(int nt) {
  return (size_t)(nt / 64) * sizeof(unsigned long long) + (size_t)kOrderBins * sizeof(int32_t) * (1 + nt / 64);
}

template <int NT>
__device__ void order_blocks(const Dev& d, const CgScal* __restrict__ scal, TeamSlot* __restrict__ fmap,
                             unsigned char* sm) {
  constexpr int NW = NT / 64;
  unsigned long long* wmax = reinterpret_cast<unsigned long long*>(sm);
  int32_t* base = reinterpret_cast<int32_t*>(wmax + NW);
  int32_t(*wcnt)[kOrderBins] = reinterpret_cast<int32_t(*)[kOrderBins]>(base + kOrderBins);
  const int n = d.geo.n_sub;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  auto cost = [&](int s) -> unsigned long long {
    const SubDesc& sd = d.subs[s];
    const unsigned long long nodes = (unsigned long long)sd.n[0] * sd.n[1] * sd.n[2];
    return (unsigned long long)(max(scal[s].iters, 0) + 1) * nodes;
  };
  // the first chunk's costs stay in registers (one subdomain per thread for
  // up to NT subdomains: each cost is read once)
  const unsigned long long cost0 = tid < n ? cost(tid) : 0ull;
  unsigned long long m = max(cost0, 1ull);
  for (int s = tid + NT; s < n; s += NT) m = max(m, cost(s));
  for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, o, 64));
  if (tid < kOrderBins) base[tid] = 0;
  if (lane == 0) wmax[w] = m;
  __syncthreads();
  unsigned long long mx = 1;
  for (int i = 0; i < NW; ++i) mx = max(mx, wmax[i]);
  const double bsc = double(kOrderBins - 1) / double(mx);
  auto bin_of = [&](unsigned long long c) { return kOrderBins - 1 - min((int)(double(c) * bsc), kOrderBins - 1); };
  auto bin = [&](int s) { return bin_of(s == tid ? cost0 : cost(s)); };
  for (int s = tid; s < n; s += NT) atomicAdd(&base[bin(s)], 1);
  __syncthreads();
  if (tid == 0) {  // counts -> first position of each bin
    int acc = 0;
    for (int k = 0; k < kOrderBins; ++k) {
      const int c = base[k];
      base[k] = acc;
      acc += c;
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += NT) {
    const int s = c0 + tid;
    const int k = s < n ? bin(s) : -1;
    wcnt[w][lane] = 0;
    __syncthreads();
    // rank among the lanes of this wave with the same bin, and the wave's count per bin
    int rank = 0;
    unsigned long long todo = __ballot(k >= 0);
    while (todo) {
      const int kk = __shfl(k, __builtin_ctzll(todo), 64);
      const unsigned long long same = __ballot(k == kk);
      if (k == kk) rank = __popcll(same & ((1ull << lane) - 1ull));
      if (lane == 0) wcnt[w][kk] = __popcll(same);
      todo &= ~same;
    }
    __syncthreads();
    if (tid < kOrderBins) {  // per bin: first position of each wave's lanes, then the next chunk's
      int acc = base[tid];
      for (int i = 0; i < NW; ++i) {
        const int c = wcnt[i][tid];
        wcnt[i][tid] = acc;
        acc += c;
      }
      base[tid] = acc;
    }
    __syncthreads();
    if (k >= 0) fmap[wcnt[w][k] + rank] = TeamSlot{s, 0, 1, 0};
    __syncthreads();
  }
}

__global__ __launch_bounds__(kOrderThreads) void k_order_blocks(Dev d, const CgScal* __restrict__ scal,
                                                                TeamSlot* __restrict__ fmap) {
  __shared__ __align__(16) unsigned char sm[order_lds_bytes(kOrderThreads)];
  order_blocks<kOrderThreads>(d, scal, fmap, sm);
}

// Every shell node of the block's planes (the state of a run's first
// residual: lambda may have been set from outside).
__global__ void __launch_bounds__(1024) k_shell_rhs(Dev d, const BlockDesc* blocks, const double* __restrict__ f,
                                                    const double* __restrict__ lam, double* __restrict__ b,
                                                    double* __restrict__ fx, double* __restrict__ bx) {
  const BlockDesc bd = blocks[blockIdx.x];
  shell_rhs(d, d.subs[bd.s], bd.z0, bd.z1, f, lam, b, fx, bx);
}

// ---------------------------------------------------------------------------- exchange

// Position of face F's nodes in the concatenated local vectors: node (a, b)
// of the face (first tangential axis fastest) is at base + a sa + b sb.
// One block per (interface pair, band of face rows): both sides' face values
// are gathered once into zero-padded LDS tiles (two halo rows and columns: the
// tangential 1D rows reach +-2), then
//   lambda_{s<-j} <- -lambda_{j<-s} + (A_sj + A_js) u_j,
//   lambda_{j<-s} <- -lambda_{s<-j} + (A_sj + A_js) u_s,   A = p M_F + q K_F,
// with M_F = Ma (x) Mb and K_F = Ka (x) Mb + Ma (x) Kb (plain 1D factors). The
// pair's geometry comes resolved from the host (one descriptor load), and the
// old lambda of a thread's first node is loaded together with the gather.
// With b given, the new data also go into both sides' right-hand sides at the
// face nodes, b = f + lambda (bx = fx + lambda for a side whose face is
// normal to its local axis 0): exact wherever a node lies on this face alone;
// the residual kernel rewrites the edge and corner nodes, where several faces'
// data add (two exchange blocks may write such a node first).
// With fmap given, grid row 0 is the block ordering for the fused kernel's
// next launch (its first block; the row's others exit), which reads only what
// the fused kernel wrote, and the pairs take rows 1 and up: the ordering runs
// beside the exchange instead of before it.
__global__ void __launch_bounds__(kExThreads) k_exchange(const ExPair* __restrict__ pairs, int rows_max,
                                                         const double* __restrict__ u, double* __restrict__ lam,
                                                         const double* __restrict__ f, double* __restrict__ b,
                                                         const double* __restrict__ fx, double* __restrict__ bx,
                                                         Dev d, const CgScal* __restrict__ scal,
                                                         TeamSlot* __restrict__ fmap) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* Us = reinterpret_cast<double*>(smem);
  int pair = blockIdx.y;
  if (fmap) {
    if (pair == 0) {
      if (blockIdx.x == 0) order_blocks<kExThreads>(d, scal, fmap, smem);
      return;
    }
    --pair;
  }
  const ExPair P = pairs[pair];
  const int na = P.na, nb = P.nb;
  const int b0 = blockIdx.x * rows_max;
  if (b0 >= nb) return;
  const int rows = min(rows_max, nb - b0);
  const int W = na + 4, H = rows + 4;
  double* Uj = Us + W * H;
  const int t0 = threadIdx.x;
  // right-hand side of face node t of the band on side s and on side j: in
  // the x-boundary arrays for a face normal to the side's local axis 0
  const bool xs = P.xb_s >= 0, xj = P.xb_j >= 0;
  const double* fs_ = xs ? fx + P.xb_s : f + P.base_s;
  const double* fj_ = xj ? fx + P.xb_j : f + P.base_j;
  double* bs_ = xs ? bx + P.xb_s : b + P.base_s;
  double* bj_ = xj ? bx + P.xb_j : b + P.base_j;
  const int64_t sas = xs ? P.xsa_s : P.sa_s, sbs = xs ? P.xsb_s : P.sb_s;
  const int64_t saj = xj ? P.xsa_j : P.sa_j, sbj = xj ? P.xsb_j : P.sb_j;
  auto node_s = [&](int t) { return (t % na) * sas + (b0 + t / na) * sbs; };
  auto node_j = [&](int t) { return (t % na) * saj + (b0 + t / na) * sbj; };
  double lf0 = 0.0, lg0 = 0.0, fs0 = 0.0, fj0 = 0.0;
  if (t0 < na * rows) {
    const int64_t t2 = (t0 % na) + (int64_t)na * (b0 + t0 / na);
    lf0 = lam[P.lam_f + t2];
    lg0 = lam[P.lam_g + t2];
    if (b) {
      fs0 = fs_[node_s(t0)];
      fj0 = fj_[node_j(t0)];
    }
  }
  for (int e = threadIdx.x; e < W * H; e += blockDim.x) {
    const int a = e % W - 2, b = e / W + b0 - 2;
    double vs = 0.0, vj = 0.0;
    if (a >= 0 && a < na && b >= 0 && b < nb) {
      vs = u[P.base_s + a * P.sa_s + b * P.sb_s];
      vj = u[P.base_j + a * P.sa_j + b * P.sb_j];
    }
    Us[e] = vs;
    Uj[e] = vj;
  }
  __syncthreads();
  // (A_sj + A_js) u_s and (A_sj + A_js) u_j at face node t of the band
  auto apply = [&](int t, double& as, double& aj) {
    const int a = t % na, b = b0 + t / na;
    const Row<double> ra = row_of<double>(a + P.kla, P.nea, P.ksa, P.msa, 0.0, 0.0);
    const Row<double> rb = row_of<double>(b + P.klb, P.neb, P.ksb, P.msb, 0.0, 0.0);
    const double ma[5] = {ra.m2, 2.0 * P.msa, ra.m0, 2.0 * P.msa, ra.m2};
    const double ka[5] = {ra.k2, -8.0 * P.ksa, ra.k0, -8.0 * P.ksa, ra.k2};
    const double mb[5] = {rb.m2, 2.0 * P.msb, rb.m0, 2.0 * P.msb, rb.m2};
    const double kb[5] = {rb.k2, -8.0 * P.ksb, rb.k0, -8.0 * P.ksb, rb.k2};
    as = 0.0;
    aj = 0.0;
#pragma unroll
    for (int ob = 0; ob < 5; ++ob) {
      const double* rs = Us + (b - b0 + ob) * W + a;
      const double* rj = Uj + (b - b0 + ob) * W + a;
      double ms_ = 0.0, ks_ = 0.0, mj = 0.0, kj = 0.0;
#pragma unroll
      for (int oa = 0; oa < 5; ++oa) {
        ms_ += ma[oa] * rs[oa];
        ks_ += ka[oa] * rs[oa];
        mj += ma[oa] * rj[oa];
        kj += ka[oa] * rj[oa];
      }
      as += P.cp * mb[ob] * ms_ + P.cq * (kb[ob] * ms_ + mb[ob] * ks_);
      aj += P.cp * mb[ob] * mj + P.cq * (kb[ob] * mj + mb[ob] * kj);
    }
    return (int64_t)a + (int64_t)na * b;
  };
  if (t0 < na * rows) {
    double as, aj;
    const int64_t t2 = apply(t0, as, aj);
    const double ls = -lg0 + aj, lj = -lf0 + as;
    lam[P.lam_f + t2] = ls;
    lam[P.lam_g + t2] = lj;
    if (b) {
      bs_[node_s(t0)] = fs0 + ls;
      bj_[node_j(t0)] = fj0 + lj;
    }
  }
  for (int t = t0 + blockDim.x; t < na * rows; t += blockDim.x) {
    double as, aj;
    const int64_t t2 = apply(t, as, aj);
    const double lf = lam[P.lam_f + t2];
    const double lg = lam[P.lam_g + t2];
    const double ls = -lg + aj, lj = -lf + as;
    lam[P.lam_f + t2] = ls;
    lam[P.lam_g + t2] = lj;
    if (b) {
      bs_[node_s(t)] = fs_[node_s(t)] + ls;
      bj_[node_j(t)] = fj_[node_j(t)] + lj;
    }
  }
}

// ---------------------------------------------------------------------------- glue and residual

// Element a (0, 1, 2: a run-time value) of a three-element set, by selects:
// indexing a private array with a run-time index would put it in scratch
// memory.
__device__ __forceinline__ int pick3(int a, int v0, int v1, int v2) { return a == 0 ? v0 : (a == 1 ? v1 : v2); }

// Global node index (per global axis) of local node (i, j, k) of sd.
__device__ __forceinline__ void global_node(const SubDesc& sd, int i, int j, int k, int& g0, int& g1, int& g2) {
  g0 = sd.lo[0] + pick3(sd.iperm[0], i, j, k);
  g1 = sd.lo[1] + pick3(sd.iperm[1], i, j, k);
  g2 = sd.lo[2] + pick3(sd.iperm[2], i, j, k);
}

// Visit the subdomain copies of local node (i, j, k) of sd in ascending
// subdomain order: fn(index of the copy in the concatenated local layout).
// Along every global axis the node has one copy, or two where it lies on an
// interface plane (the lower subdomain's first); each copy's local index
// follows from the global node through that subdomain's own axis order.
template <class Fn>
__device__ __forceinline__ int for_copies(const Dev& d, const SubDesc& sd, int i, int j, int k, Fn&& fn) {
  int g0, g1, g2;
  global_node(sd, i, j, k, g0, g1, g2);
  int p0[3], nc[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int a = sd.iperm[g];
    const int la = pick3(a, i, j, k), na = pick3(a, sd.n[0], sd.n[1], sd.n[2]);
    const int flo = pick3(a, sd.face[0], sd.face[2], sd.face[4]), fhi = pick3(a, sd.face[1], sd.face[3], sd.face[5]);
    nc[g] = 1;
    p0[g] = sd.pidx[g];
    if (la == 0 && flo >= 0) {
      nc[g] = 2;
      p0[g] = sd.pidx[g] - 1;
    } else if (la == na - 1 && fhi >= 0) {
      nc[g] = 2;
    }
  }
  const int Px = d.geo.nparts[0], Py = d.geo.nparts[1];
  for (int cz = 0; cz < nc[2]; ++cz)
    for (int cy = 0; cy < nc[1]; ++cy)
      for (int cx = 0; cx < nc[0]; ++cx) {
        const int s2 = sd.sbase + (p0[0] + cx) + Px * ((p0[1] + cy) + Py * (p0[2] + cz));
        const SubDesc& o = d.subs[s2];
        // the node's local coordinates in o: its global ones along o's axes
        const int l0 = pick3(o.perm[0], g0 - o.lo[0], g1 - o.lo[1], g2 - o.lo[2]);
        const int l1 = pick3(o.perm[1], g0 - o.lo[0], g1 - o.lo[1], g2 - o.lo[2]);
        const int l2 = pick3(o.perm[2], g0 - o.lo[0], g1 - o.lo[1], g2 - o.lo[2]);
        fn(o.off + l0 + (int64_t)o.n[0] * (l1 + (int64_t)o.n[1] * l2));
      }
  return nc[0] * nc[1] * nc[2];
}

// Global residual check (Sec. 6 stops on it) in three passes over the local
// layout. Only nodes on a subdomain's shell have more than one copy.
__device__ __forceinline__ bool on_shell(const SubDesc& sd, int i, int j, int k) {
  return i == 0 || j == 0 || k == 0 || i == sd.n[0] - 1 || j == sd.n[1] - 1 || k == sd.n[2] - 1;
}
// A node on an interface belongs to the copy that is not at the lower end of
// any interface.
__device__ __forceinline__ bool owns_node(const SubDesc& sd, int i, int j, int k) {
  return !((i == 0 && sd.face[0] >= 0) || (j == 0 && sd.face[2] >= 0) || (k == 0 && sd.face[4] >= 0));
}
// Shell node t of sd (t < shell_nodes): the first and last planes, then the
// ring of each plane in between (every node, in layout order, when some axis
// has at most 2 nodes).
__device__ __forceinline__ void shell_node(const SubDesc& sd, int t, int& i, int& j, int& k) {
  const int nx = sd.n[0], ny = sd.n[1], nz = sd.n[2];
  const int plane = nx * ny, ring = 2 * (nx + ny) - 4;
  if (nx <= 2 || ny <= 2 || nz <= 2) {
    k = t / plane;
    j = (t - k * plane) / nx;
    i = t - k * plane - j * nx;
  } else if (t < 2 * plane) {
    k = t < plane ? 0 : nz - 1;
    const int e = t < plane ? t : t - plane;
    j = e / nx;
    i = e - j * nx;
  } else {
    const int e = t - 2 * plane;
    k = 1 + e / ring;
    const int r = e - (k - 1) * ring;
    if (r < nx) {
      i = r;
      j = 0;
    } else if (r < 2 * nx) {
      i = r - nx;
      j = ny - 1;
    } else {
      const int r2 = r - 2 * nx;  // the two side columns, rows 1 .. ny-2
      i = r2 < ny - 2 ? 0 : nx - 1;
      j = 1 + (r2 < ny - 2 ? r2 : r2 - (ny - 2));
    }
  }
}

// First pass: u~ (the average of the node's copies) at every shell node.
__global__ void k_glue_shell(Dev d, const double* __restrict__ u, double* __restrict__ ut) {
  const SubDesc sd = d.subs[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= shell_nodes(sd.n[0], sd.n[1], sd.n[2])) return;
  int i, j, k;
  shell_node(sd, t, i, j, k);
  double s = 0.0;
  const int n = for_copies(d, sd, i, j, k, [&](int64_t idx) { s += u[idx]; });
  ut[sd.off + i + (int64_t)sd.n[0] * (j + (int64_t)sd.n[1] * k)] = s / double(n);
}

// Second pass, the z-march of rho = f - K^N u~ (K^N: the local stiffness
// without Robin terms), u~ read from the first pass on the shell and from u
// inside. An interior node has one copy and is owned: its rho^2 and f^2 go
// straight into the block's sums. A shell node's rho is stored for the third
// pass, which sums the copies. The owner of each node writes u~ to phi when
// phi is given. ZU: every block marches one segment (the host checks;
// otherwise the partials are NaN and the check reports a breakdown).
template <int CPT, bool PHI, bool ZU = false>
__global__ void __launch_bounds__(Bound<CPT>::value)
    k_check_residual(Dev d, const BlockDesc* blocks, const double* __restrict__ u, const double* __restrict__ ut,
                     const double* __restrict__ f, double* __restrict__ rho, double* __restrict__ phi,
                     double* __restrict__ part) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* lds = reinterpret_cast<double*>(smem);
  const BlockDesc bd = blocks[blockIdx.x];
  const SubDesc sd = d.subs[bd.s];
  Slots<double, CPT, false> sl;
  slots_init(sl, sd, d.geo, bd.z0, bd.z1, false);
  lds_zero(lds, sl.G * kPlanes * sl.SP);
  __syncthreads();
  const double* __restrict__ ub = u + sl.off;
  const double* __restrict__ utb = ut + sl.off;
  const double* __restrict__ fb = f + sl.off;
  double* __restrict__ rhob = rho + sl.off;
  // plain scalars only in the functors (a descriptor captured whole would be
  // kept in scratch memory)
  const int nx1 = sd.n[0] - 1, ny1 = sd.n[1] - 1, nz1 = sd.n[2] - 1;
  const bool fx = sd.face[0] >= 0, fy = sd.face[2] >= 0, fz = sd.face[4] >= 0;
  auto shell = [=](int i, int j, int k) { return i == 0 || j == 0 || k == 0 || i == nx1 || j == ny1 || k == nz1; };
  // the operand u~ is prefetched with the ring; f is loaded when its plane's
  // operand is made and carried to the store two steps later (a load in the
  // store itself would wait for every load in flight)
  auto fetch = [=](uint32_t li, bool, int i, int j, int k) { return at(shell(i, j, k) ? utb : ub, li); };
  auto make = [=](double v, uint32_t li, bool, bool, double) { return OpCarry<double>{v, at(fb, li)}; };
  // phi index of local node (i, j, k): the global node through the axis order
  const int64_t nn0 = d.geo.nn[0], nn01 = (int64_t)d.geo.nn[0] * d.geo.nn[1];
  const int64_t pbase = sd.copy * nn01 * d.geo.nn[2] + sd.lo[0] + nn0 * sd.lo[1] + nn01 * sd.lo[2];
  const int64_t st0 = sd.perm[0] == 0 ? 1 : (sd.perm[0] == 1 ? nn0 : nn01);
  const int64_t st1 = sd.perm[1] == 0 ? 1 : (sd.perm[1] == 1 ? nn0 : nn01);
  const int64_t st2 = sd.perm[2] == 0 ? 1 : (sd.perm[2] == 1 ? nn0 : nn01);
  double arr = 0.0, aff = 0.0;
  auto store = [&](uint32_t li, bool en, bool, int i, int j, int k, double q, double fv, double) {
    if (!en) return;
    const double rv = fv - q;
    const bool sh = shell(i, j, k);
    if (sh) {
      at(rhob, li) = rv;
    } else {
      arr += rv * rv;
      aff += fv * fv;
    }
    // the glued solution, when asked for (once per solve): u~ read again
    if constexpr (PHI) {
      if (!((i == 0 && fx) || (j == 0 && fy) || (k == 0 && fz)))
        phi[pbase + i * st0 + j * st1 + k * st2] = at(sh ? utb : ub, li);
    }
  };
  const bool badseg = ZU && sl.G != 1;
  if (!badseg) zmarch<ZU>(sl, lds, fetch, make, store);
  double acc[2] = {arr, aff};
  block_sum(acc);
  if (badseg) acc[0] = acc[1] = __builtin_nan("");
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = acc[0];
    part[2 * blockIdx.x + 1] = acc[1];
  }
}

// Third pass: the owned shell nodes of every subdomain, rho and f summed over
// the node's copies and squared into the block's sums.
__global__ void k_assemble_shell(Dev d, const double* __restrict__ rho, const double* __restrict__ f,
                                 double* __restrict__ part) {
  const SubDesc sd = d.subs[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (t < shell_nodes(sd.n[0], sd.n[1], sd.n[2])) {
    int i, j, k;
    shell_node(sd, t, i, j, k);
    if (owns_node(sd, i, j, k)) {
      double rs = 0.0, fs = 0.0;
      for_copies(d, sd, i, j, k, [&](int64_t idx) {
        rs += rho[idx];
        fs += f[idx];
      });
      acc[0] = rs * rs;
      acc[1] = fs * fs;
    }
  }
  block_sum(acc);
  if (threadIdx.x == 0) {
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = acc[0];
    part[2 * b + 1] = acc[1];
  }
}

// Per copy: res_c = ||f - K u~|| / ||f|| from the sums of both passes (the
// first pass's partials part[0 .. na), the second's part[na .. na + nb); the
// blocks of copy c are the c-th of `copies` equal contiguous ranges of each),
// and the largest over the copies (the stopping quantity). dev_out: [max res,
// r'r, f'f of the worst copy, res_0 .. res_{copies-1}].
__global__ void k_final_norm(const double* __restrict__ part, int na, int nb, int copies, const int32_t* flags,
                             double* dev_out, double* host_out) {
  const int pa = na / copies, pb = nb / copies;
  double worst = 0.0, wr = 0.0, wf = 0.0;
  for (int c = 0; c < copies; ++c) {
    double acc[2] = {0.0, 0.0};
    for (int b = c * pa + threadIdx.x; b < (c + 1) * pa; b += blockDim.x) {
      acc[0] += part[2 * b];
      acc[1] += part[2 * b + 1];
    }
    for (int b = na + c * pb + threadIdx.x; b < na + (c + 1) * pb; b += blockDim.x) {
      acc[0] += part[2 * b];
      acc[1] += part[2 * b + 1];
    }
    block_sum(acc);
    const double res = acc[1] > 0.0 ? sqrt(acc[0] / acc[1]) : (acc[0] > 0.0 ? INFINITY : 0.0);
    if (threadIdx.x == 0) dev_out[3 + c] = res;
    if (c == 0 || !(res <= worst)) {  // NaN propagates
      worst = res;
      wr = acc[0];
      wf = acc[1];
    }
  }
  if (threadIdx.x == 0) {
    dev_out[0] = worst;
    dev_out[1] = wr;
    dev_out[2] = wf;
    if (host_out) {
      host_out[0] = worst;
      host_out[1] = flags ? double(*flags) : 0.0;
    }
  }
}

__global__ void k_fill(double* x, int64_t n, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ---------------------------------------------------------------------------- loads

// f_s = 4 pi G sum over the elements of s containing the node of drho_e * prod_d w_d,
// w = h/6 at an element end, 2h/3 at its mid-point.
__global__ void k_load_density(Dev d, const double* __restrict__ drho, double G, double* __restrict__ f) {
  const SubDesc sd = d.subs[blockIdx.y];
  const int n = sd.n[0] * sd.n[1] * sd.n[2];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int gn[3];
  global_node(sd, t % sd.n[0], (t / sd.n[0]) % sd.n[1], t / (sd.n[0] * sd.n[1]), gn[0], gn[1], gn[2]);
  int el[3][2], ne[3];
  double w[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {  // global axis a
    const int gc = gn[a];
    const int e0 = sd.e0[a], e1 = sd.e0[a] + pick3(sd.iperm[a], sd.ne2[0], sd.ne2[1], sd.ne2[2]) / 2;
    const double h = d.geo.h[a];
    ne[a] = 0;
    if (gc & 1) {
      el[a][0] = (gc - 1) / 2;
      w[a][0] = 2.0 * h / 3.0;
      ne[a] = 1;
    } else {
      const int lo = gc / 2 - 1, hi = gc / 2;
      if (lo >= e0 && lo < e1) {
        el[a][ne[a]] = lo;
        w[a][ne[a]] = h / 6.0;
        ++ne[a];
      }
      if (hi >= e0 && hi < e1) {
        el[a][ne[a]] = hi;
        w[a][ne[a]] = h / 6.0;
        ++ne[a];
      }
    }
  }
  const int Ex = d.geo.ne[0], Ey = d.geo.ne[1];
  double acc = 0.0;
  for (int cz = 0; cz < ne[2]; ++cz)
    for (int cy = 0; cy < ne[1]; ++cy)
      for (int cx = 0; cx < ne[0]; ++cx)
        acc += drho[el[0][cx] + (int64_t)Ex * (el[1][cy] + (int64_t)Ey * el[2][cz])] * (w[0][cx] * w[1][cy] * w[2][cz]);
  f[sd.off + t] = 4.0 * M_PI * G * acc;
}

__global__ void k_load_nodes(Dev d, const double* __restrict__ fn, double* __restrict__ f) {
  const SubDesc sd = d.subs[blockIdx.y];
  const int n = sd.n[0] * sd.n[1] * sd.n[2];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int li[3] = {t % sd.n[0], (t / sd.n[0]) % sd.n[1], t / (sd.n[0] * sd.n[1])};
  int mult = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if ((li[a] == 0 && sd.face[2 * a] >= 0) || (li[a] == sd.n[a] - 1 && sd.face[2 * a + 1] >= 0)) mult *= 2;
  int g0, g1, g2;
  global_node(sd, li[0], li[1], li[2], g0, g1, g2);
  const int64_t g = g0 + (int64_t)d.geo.nn[0] * (g1 + (int64_t)d.geo.nn[1] * g2);
  f[sd.off + t] = fn[g] / double(mult);
}

// dJ/ddrho_e = 4 pi G sum over the 27 nodes a of e of psi_a int_e phi_a, the
// transpose of the density-to-load map (w = h/6, 2h/3, h/6 per axis).
__global__ void k_grad_density(Geom g, const double* __restrict__ psi, double G, double* __restrict__ grad) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t ne = (int64_t)g.ne[0] * g.ne[1] * g.ne[2];
  if (e >= ne) return;
  const int ex = int(e % g.ne[0]);
  const int ey = int((e / g.ne[0]) % g.ne[1]);
  const int ez = int(e / ((int64_t)g.ne[0] * g.ne[1]));
  const double wx[3] = {g.h[0] / 6.0, 2.0 * g.h[0] / 3.0, g.h[0] / 6.0};
  const double wy[3] = {g.h[1] / 6.0, 2.0 * g.h[1] / 3.0, g.h[1] / 6.0};
  const double wz[3] = {g.h[2] / 6.0, 2.0 * g.h[2] / 3.0, g.h[2] / 6.0};
  double acc = 0.0;
#pragma unroll
  for (int az = 0; az < 3; ++az)
#pragma unroll
    for (int ay = 0; ay < 3; ++ay) {
      const int64_t row = (int64_t)g.nn[0] * ((2 * ey + ay) + (int64_t)g.nn[1] * (2 * ez + az));
      double s = 0.0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) s += wx[ax] * psi[row + 2 * ex + ax];
      acc += wy[ay] * wz[az] * s;
    }
  grad[e] = 4.0 * M_PI * G * acc;
}

// ---------------------------------------------------------------------------- launchers

hipError_t launch_grad_density(const Geom& g, const double* psi, double G, double* grad, hipStream_t st) {
  const int64_t ne = (int64_t)g.ne[0] * g.ne[1] * g.ne[2];
  hipLaunchKernelGGL(k_grad_density, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, g, psi, G, grad);
  return hipGetLastError();
}

static dim3 node_grid(const Dev& d, int max_n, int threads) { return dim3((max_n + threads - 1) / threads, d.geo.n_sub); }

hipError_t launch_load_density(const Dev& d, int max_n, const double* drho, double G, double* f_loc,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_load_density, node_grid(d, max_n, 256), dim3(256), 0, st, d, drho, G, f_loc);
  return hipGetLastError();
}

hipError_t launch_load_nodes(const Dev& d, int max_n, const double* f_nodes, double* f_loc, hipStream_t st) {
  hipLaunchKernelGGL(k_load_nodes, node_grid(d, max_n, 256), dim3(256), 0, st, d, f_nodes, f_loc);
  return hipGetLastError();
}

hipError_t launch_residual(const Dev& d, const SegLaunch& L, int fp32, bool rz, const double* u, const double* f,
                           const double* lam, double* b, double* bx, void* r_out, double* part, double* team_part,
                           hipStream_t st) {
  SOS_DISPATCH_Q(d.hasq, {
  if (fp32 && rz && L.zu) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_residual<float, C, Q, true, true>), dim3(L.nblocks),
                                               dim3(L.threads), L.lds64, st, d, L.blocks, u, f, lam, b, bx, (float*)r_out,
                                               part, team_part));
  } else if (fp32 && rz) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_residual<float, C, Q, true>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds64, st, d, L.blocks, u, f, lam, b, bx, (float*)r_out, part, team_part));
  } else if (fp32 && L.zu) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_residual<float, C, Q, false, true>), dim3(L.nblocks),
                                               dim3(L.threads), L.lds64, st, d, L.blocks, u, f, lam, b, bx, (float*)r_out, part,
                                               team_part));
  } else if (fp32) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_residual<float, C, Q, false>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds64, st, d, L.blocks, u, f, lam, b, bx, (float*)r_out, part, team_part));
  } else if (rz && L.zu) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_residual<double, C, Q, true, true>), dim3(L.nblocks),
                                               dim3(L.threads), L.lds64, st, d, L.blocks, u, f, lam, b, bx,
                                               (double*)r_out, part, team_part));
  } else if (rz) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_residual<double, C, Q, true>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds64, st, d, L.blocks, u, f, lam, b, bx, (double*)r_out, part, team_part));
  } else {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_residual<double, C, Q, false>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds64, st, d, L.blocks, u, f, lam, b, bx, (double*)r_out, part, team_part));
  }
  });
  return hipGetLastError();
}

hipError_t launch_cg_init(const Dev& d, const SegLaunch& L, const double* part, double tol_rel, double tol_abs,
                          CgScal* scal, int32_t* ndone, hipStream_t st) {
  const int n = d.geo.n_sub;
  hipLaunchKernelGGL(k_cg_init, dim3((n + 255) / 256), dim3(256), 0, st, n, L.bfirst, part, tol_rel, tol_abs,
                     scal, ndone);
  return hipGetLastError();
}

hipError_t launch_cg_apply(const Dev& d, const SegLaunch& L, int fp32, int t, int max_inner, const void* r,
                           const void* p_old, void* p_new, void* q, double* part, CgScal* scal, int32_t* ndone,
                           unsigned long long* counters, int32_t* flags, hipStream_t st) {
  SOS_DISPATCH_Q(d.hasq, {
  if (fp32 && L.zu) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_cg_apply<float, C, Q, true>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds32, st, d, L.blocks, L.bfirst, t, max_inner, (const float*)r,
                                               (const float*)p_old, (float*)p_new, (float*)q, part, scal, ndone,
                                               counters, flags));
  } else if (fp32) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_cg_apply<float, C, Q>), dim3(L.nblocks), dim3(L.threads), L.lds32,
                                               st, d, L.blocks, L.bfirst, t, max_inner, (const float*)r,
                                               (const float*)p_old, (float*)p_new, (float*)q, part, scal, ndone,
                                               counters, flags));
  } else if (L.zu) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_cg_apply<double, C, Q, true>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds64, st, d, L.blocks, L.bfirst, t, max_inner, (const double*)r,
                                               (const double*)p_old, (double*)p_new, (double*)q, part, scal,
                                               ndone, counters, flags));
  } else {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_cg_apply<double, C, Q>), dim3(L.nblocks), dim3(L.threads), L.lds64,
                                               st, d, L.blocks, L.bfirst, t, max_inner, (const double*)r,
                                               (const double*)p_old, (double*)p_new, (double*)q, part, scal,
                                               ndone, counters, flags));
  }
  });
  return hipGetLastError();
}

hipError_t launch_cg_update(const Dev& d, const SegLaunch& L, int fp32, int t, void* x, const void* p, void* r,
                            const void* q, double* part, CgScal* scal, int32_t* ndone, int32_t* flags,
                            hipStream_t st) {
  SOS_DISPATCH_Q(d.hasq, {
  if (fp32) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_cg_update<float, C, Q>), dim3(L.nblocks), dim3(L.threads), 0, st, d,
                                               L.blocks, L.bfirst, t, (float*)x, (const float*)p, (float*)r,
                                               (const float*)q, part, scal, ndone, flags));
  } else {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_cg_update<double, C, Q>), dim3(L.nblocks), dim3(L.threads), 0, st, d,
                                               L.blocks, L.bfirst, t, (double*)x, (const double*)p, (double*)r,
                                               (const double*)q, part, scal, ndone, flags));
  }
  });
  return hipGetLastError();
}

hipError_t launch_add_correction(const Dev& d, const SegLaunch& L, int fp32, double* u, const void* x,
                                 const CgScal* scal, hipStream_t st) {
  if (fp32) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_add_correction<float, C>), dim3(L.nblocks), dim3(L.threads), 0,
                                               st, d, L.blocks, u, (const float*)x, scal));
  } else {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_add_correction<double, C>), dim3(L.nblocks), dim3(L.threads), 0,
                                               st, d, L.blocks, u, (const double*)x, scal));
  }
  return hipGetLastError();
}

hipError_t launch_fused_cg(const Dev& d, const SegLaunch& L, int fp32, int threads, int cpt, size_t lds,
                           const FusedArgs& a, hipStream_t st, bool* plain) {
  if (a.res && (!fp32 || !a.zu || lds > a.lds_bytes)) return hipErrorInvalidValue;
  SOS_DISPATCH_CPT(cpt, return launch_fused_cpt<C>(d, L, fp32, threads, lds, a, st, plain));
  return hipSuccess;
}

hipError_t launch_order_blocks(const Dev& d, const CgScal* scal, TeamSlot* fmap, hipStream_t st) {
  hipLaunchKernelGGL(k_order_blocks, dim3(1), dim3(kOrderThreads), 0, st, d, scal, fmap);
  return hipGetLastError();
}

hipError_t launch_exchange(const ExPair* pairs, int32_t n_pairs, int32_t max_na, int32_t max_nb, const double* u,
                           double* lam, const double* f, double* b, const double* fx, double* bx, hipStream_t st,
                           const Dev* d, const CgScal* scal, TeamSlot* fmap) {
  if (n_pairs == 0) return fmap ? launch_order_blocks(*d, scal, fmap, st) : hipSuccess;
  if ((fmap && (!d || !scal)) || (b && (!f || !fx || !bx))) return hipErrorInvalidValue;
  const int rows = exchange_rows(max_na);
  size_t lds = 2 * sizeof(double) * (size_t)(max_na + 4) * (size_t)(rows + 4);
  if (fmap) lds = std::max(lds, order_lds_bytes(kExThreads));
  hipLaunchKernelGGL(k_exchange, dim3((max_nb + rows - 1) / rows, n_pairs + (fmap ? 1 : 0)), dim3(kExThreads), lds, st,
                     pairs, rows, u, lam, f, b, fx, bx, fmap ? *d : Dev{}, scal, fmap);
  return hipGetLastError();
}

hipError_t launch_shell_rhs(const Dev& d, const SegLaunch& L, const double* f, const double* lam, double* b,
                            double* fx, double* bx, hipStream_t st) {
  hipLaunchKernelGGL(k_shell_rhs, dim3(L.nblocks), dim3(L.threads), 0, st, d, L.blocks, f, lam, b, fx, bx);
  return hipGetLastError();
}

hipError_t launch_glue_shell(const Dev& d, int max_shell, const double* u, double* ut, hipStream_t st) {
  hipLaunchKernelGGL(k_glue_shell, node_grid(d, max_shell, kAssembleThreads), dim3(kAssembleThreads), 0, st, d, u,
                     ut);
  return hipGetLastError();
}

hipError_t launch_check_residual(const Dev& d, const SegLaunch& L, const double* u, const double* ut,
                                 const double* f, double* rho, double* phi, double* part, hipStream_t st) {
  if (phi && L.zu) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_check_residual<C, true, true>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds64, st, d, L.blocks, u, ut, f, rho, phi, part));
  } else if (phi) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_check_residual<C, true>), dim3(L.nblocks), dim3(L.threads), L.lds64,
                                               st, d, L.blocks, u, ut, f, rho, phi, part));
  } else if (L.zu) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_check_residual<C, false, true>), dim3(L.nblocks), dim3(L.threads),
                                               L.lds64, st, d, L.blocks, u, ut, f, rho, phi, part));
  } else {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_check_residual<C, false>), dim3(L.nblocks), dim3(L.threads), L.lds64,
                                               st, d, L.blocks, u, ut, f, rho, phi, part));
  }
  return hipGetLastError();
}

int shell_blocks(const Dev& d, int max_shell) {
  return ((max_shell + kAssembleThreads - 1) / kAssembleThreads) * d.geo.n_sub;
}

hipError_t launch_assemble_shell(const Dev& d, int max_shell, const double* rho, const double* f, double* part,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_assemble_shell, node_grid(d, max_shell, kAssembleThreads), dim3(kAssembleThreads), 0, st, d,
                     rho, f, part);
  return hipGetLastError();
}

hipError_t launch_final_norm(const double* part, int32_t na, int32_t nb, int32_t copies, const int32_t* flags,
                             double* dev_out, double* host_out, hipStream_t st) {
  hipLaunchKernelGGL(k_final_norm, dim3(1), dim3(1024), 0, st, part, na, nb, copies, flags, dev_out, host_out);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}

hipError_t launch_apply(const Dev& d, const SegLaunch& L, int fp32, const void* x, void* y, hipStream_t st) {
  SOS_DISPATCH_Q(d.hasq, {
  if (fp32) {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_apply<float, C, Q>), dim3(L.nblocks), dim3(L.threads), L.lds32, st, d,
                                               L.blocks, (const float*)x, (float*)y));
  } else {
    SOS_DISPATCH_CPT(L.cpt, hipLaunchKernelGGL((k_apply<double, C, Q>), dim3(L.nblocks), dim3(L.threads), L.lds64, st,
                                               d, L.blocks, (const double*)x, (double*)y));
  }
  });
  return hipGetLastError();
}

}  // namespace sos
