// Device code shared by the translation units of the HIP library: the z-march
// operator, the reductions, the team barrier and the kernel templates.
//
// Operator. On a subdomain box the Robin-augmented Q2 stiffness is the
// Kronecker sum of 1D factors (tensor-product elements, Sec. 3 operator p on
// interface ends):
//   A = Kx' (x) My (x) Mz + Mx (x) Ky' (x) Mz + Mx (x) My (x) Kz',
// K' = K + diag(p at interface ends). It is applied matrix-free, marching over
// the z-planes of the subdomain: every x-y plane of the input is staged in a
// zero-padded LDS plane, reduced along y (u = My p, v = Ky' p) and then along x
// (S = Kx' u + Mx v, T = Mx u), and each plane's (S, T) is scattered into a
// ring of five z-accumulators held in registers:
//   q_k = sum_k' Mz[k][k'] S_k' + Kz'[k][k'] T_k'.
// About 30 flops per node, no MFMA: the path is bound by memory traffic.
//
// 1D rows of the assembled Q2 matrices on an interval of ne elements (closure
// nodes 0..2ne): stiffness (1/(3h)) x {1,-8,14,-8,1} at interior vertices,
// {-8,16,-8} at mid-points, {7,-8,1} / {1,-8,7} at the two ends; mass
// (h/30) x {-1,2,8,2,-1}, {2,16,2}, {4,2,-1}, {-1,2,4}. The +-1 entries are
// the same in every row, the +-2 entries are those of a vertex row or zero, so
// only the centre entry depends on the node type. Neighbours outside the
// subdomain's unknowns read the zero padding of the LDS plane (x, y) or feed
// outputs outside the subdomain that are never stored (z).
//
// CG (Sec. 6: diagonal preconditioner). Each iteration is two passes:
//   A: p = D^-1 r + beta p_old (recomputed on halo planes), q = A p, p'q
//   B: x += alpha p, r -= alpha q, r'z, r'r  (pointwise)
// Reductions are wave64 shuffles, then a fixed-order sum over waves and over
// the blocks of a subdomain: results are bitwise repeatable.
#pragma once

#include "sos_kernels.h"

#include <math.h>

#include <type_traits>

namespace sos {


// Element li of an array whose base is uniform across the wavefront, addressed
// with a 32-bit byte offset: the base stays in scalar registers and each lane
// carries one 32-bit offset shared by all arrays indexed alike.
template <typename T>
__device__ __forceinline__ T& at(T* base, uint32_t li) {
  using C = std::conditional_t<std::is_const<T>::value, const char, char>;
  return *reinterpret_cast<T*>(reinterpret_cast<C*>(base) + li * (uint32_t)sizeof(T));
}

// Data that another workgroup of the same launch writes or reads (the halo
// planes of a team of workgroups sharing one subdomain, the team's partial
// sums) goes through agent-scope relaxed atomic loads and stores: they are
// coherent across the L2 caches of all XCDs by themselves, so the team barrier
// needs no L2 write-back or invalidation (which would also evict every other
// vector of the sweep). Ordering comes from waiting for all stores before the
// barrier arrival and from issuing these loads after it.
template <typename T>
__device__ __forceinline__ T ld_coh(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// s_waitcnt vmcnt(0): every vector memory operation of the wave has completed
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }


// ---------------------------------------------------------------------------- 1D rows

template <typename T>
struct Row {
  T k0, m0, k2, m2;  // centre and +-2 entries (the +-1 entries are -8ks, 2ms)
};

template <typename T>
__device__ __forceinline__ Row<T> row_of(int c, int ne2, T ks, T ms, T elo, T ehi) {
  Row<T> r;
  if (c & 1) {
    r.k0 = T(16) * ks;
    r.m0 = T(16) * ms;
    r.k2 = T(0);
    r.m2 = T(0);
  } else {
    r.k2 = ks;
    r.m2 = -ms;
    if (c == 0) {
      r.k0 = T(7) * ks + elo;
      r.m0 = T(4) * ms;
    } else if (c == ne2) {
      r.k0 = T(7) * ks + ehi;
      r.m0 = T(4) * ms;
    } else {
      r.k0 = T(14) * ks;
      r.m0 = T(8) * ms;
    }
  }
  return r;
}

// 0 mid-point, 1 interior vertex, 2 first closure node, 3 last closure node
__device__ __forceinline__ int row_kind(int c, int ne2) {
  return (c & 1) ? 0 : (c == 0 ? 2 : (c == ne2 ? 3 : 1));
}

// ---------------------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum N values over the block; every thread receives the sums (fixed order).
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
  __shared__ double red[N * 16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int n = 0; n < N; ++n) v[n] = wave_sum(v[n]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int n = 0; n < N; ++n) red[n * 16 + w] = v[n];
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < N; ++n) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[n * 16 + k];
    v[n] = s;
  }
}

// ---------------------------------------------------------------------------- march geometry

template <typename T, int CPT, bool Q = false>
struct Slots {
  int nx, ny, nz, S, PX, SP, G, seglen;
  int64_t off;
  int c[CPT], i[CPT], j[CPT], g[CPT], z0[CPT], z1[CPT], lp[CPT];
  int uz0, uz1;  // the block's z-range (the segment of every slot when G == 1)
  bool ra;       // wave-owned rows (G == 1): the x-pass needs no barrier
  bool act[CPT];
  T kx0[CPT], mx0[CPT], kx2[CPT], mx2[CPT];
  T ky0[CPT], my0[CPT], ky2[CPT], my2[CPT];
  T dv0[CPT], dv1[CPT], dv2[CPT], dv3[CPT];  // inverse diagonal per z row kind
  T ex[CPT], ey[CPT], qx[CPT], qy[CPT];       // Robin p and q at the column's x / y interface end
  T kx1, mx1, ky1, my1, kz1, mz1;
  int zklo, zne2;
  T zks, zms, zelo, zehi, zqlo, zqhi;
  bool hasq;                                  // any second-order face term
};

template <typename T, int CPT, bool Q>
__device__ __forceinline__ void slots_init(Slots<T, CPT, Q>& sl, const SubDesc& d, const Geom& geo, int zb0,
                                           int zb1, bool robin, bool ra = false) {
  sl.nx = d.n[0];
  sl.ny = d.n[1];
  sl.nz = d.n[2];
  sl.S = sl.nx * sl.ny;
  sl.PX = sl.nx + 2 * kPad;
  sl.SP = sl.PX * (sl.ny + 2 * kPad);
  sl.off = d.off;
  const int NT = blockDim.x;
  const int zlen = zb1 - zb0;
  // wave-owned rows: one segment, R rows per wave (the caller checks that the
  // block's waves cover the plane)
  sl.ra = ra;
  sl.G = ra ? 1 : march_segments(sl.nx, sl.ny, zlen, NT, CPT);
  const int R = ra ? ra_rows(sl.nx, CPT) : 0;
  sl.uz0 = zb0;
  sl.uz1 = zb1;
  sl.seglen = (zlen + sl.G - 1) / sl.G;
  (void)geo;
  const T ksx = T(d.ks[0]), msx = T(d.ms[0]);
  const T ksy = T(d.ks[1]), msy = T(d.ms[1]);
  sl.zks = T(d.ks[2]);
  sl.zms = T(d.ms[2]);
  sl.kx1 = T(-8) * ksx;
  sl.mx1 = T(2) * msx;
  sl.ky1 = T(-8) * ksy;
  sl.my1 = T(2) * msy;
  sl.kz1 = T(-8) * sl.zks;
  sl.mz1 = T(2) * sl.zms;
  sl.zklo = d.klo[2];
  sl.zne2 = d.ne2[2];
  sl.zelo = robin ? T(d.elo[2]) : T(0);
  sl.zehi = robin ? T(d.ehi[2]) : T(0);
  if constexpr (Q) {
    sl.zqlo = robin ? T(d.qlo[2]) : T(0);
    sl.zqhi = robin ? T(d.qhi[2]) : T(0);
    sl.hasq = robin && (d.qlo[0] > 0.0 || d.qhi[0] > 0.0 || d.qlo[1] > 0.0 || d.qhi[1] > 0.0 ||
                        d.qlo[2] > 0.0 || d.qhi[2] > 0.0);
  } else {
    sl.zqlo = sl.zqhi = T(0);
    sl.hasq = false;
  }
  // centre entries of the four z row kinds (for the diagonal)
  T kz0[4], mz0[4];
  kz0[0] = T(16) * sl.zks;
  mz0[0] = T(16) * sl.zms;
  kz0[1] = T(14) * sl.zks;
  mz0[1] = T(8) * sl.zms;
  kz0[2] = T(7) * sl.zks + sl.zelo;
  mz0[2] = T(4) * sl.zms;
  kz0[3] = T(7) * sl.zks + sl.zehi;
  mz0[3] = T(4) * sl.zms;
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
    int g, col;
    bool cover;
    if (ra) {
      // slot q = lane + 64 m of wave w: row w R + q / nx, column q % nx; a
      // slot past the wave's rows or the plane takes column 0 and stays idle
      const int q = (threadIdx.x & 63) + 64 * m;
      const int rq = q / sl.nx;
      const int jr = (threadIdx.x >> 6) * R + rq;
      cover = rq < R && jr < sl.ny;
      g = 0;
      col = cover ? (q - rq * sl.nx) + sl.nx * jr : 0;
    } else {
      const int sigma = threadIdx.x + NT * m;
      g = sigma / sl.S;
      col = sigma - g * sl.S;
      cover = g < sl.G;
    }
    sl.g[m] = g;
    sl.z0[m] = zb0 + g * sl.seglen;
    sl.z1[m] = min(zb1, sl.z0[m] + sl.seglen);
    sl.act[m] = cover && (sl.z0[m] < zb1);
    sl.c[m] = col;
    const int i = col % sl.nx, j = col / sl.nx;
    sl.i[m] = i;
    sl.j[m] = j;
    sl.lp[m] = g * kPlanes * sl.SP + (i + kPad) + sl.PX * (j + kPad);
    Row<T> rx = row_of<T>(i + d.klo[0], d.ne2[0], ksx, msx, robin ? T(d.elo[0]) : T(0),
                          robin ? T(d.ehi[0]) : T(0));
    Row<T> ry = row_of<T>(j + d.klo[1], d.ne2[1], ksy, msy, robin ? T(d.elo[1]) : T(0),
                          robin ? T(d.ehi[1]) : T(0));
    sl.kx0[m] = rx.k0;
    sl.mx0[m] = rx.m0;
    sl.kx2[m] = rx.k2;
    sl.mx2[m] = rx.m2;
    sl.ky0[m] = ry.k0;
    sl.my0[m] = ry.m0;
    sl.ky2[m] = ry.k2;
    sl.my2[m] = ry.m2;
    // interface-end coefficients of this column (0/1 blends, no selects
    // between descriptor fields)
    const int cxi = i + d.klo[0], cyj = j + d.klo[1];
    const T wxl = cxi == 0 ? T(1) : T(0), wxh = cxi == d.ne2[0] ? T(1) : T(0);
    const T wyl = cyj == 0 ? T(1) : T(0), wyh = cyj == d.ne2[1] ? T(1) : T(0);
    const T rb = robin ? T(1) : T(0);
    const T a1 = rx.k0 * ry.m0 + rx.m0 * ry.k0;
    const T a2 = rx.m0 * ry.m0;
    T b1 = T(0), b2 = T(0), b3 = T(0);
    if constexpr (Q) {
      sl.ex[m] = rb * (wxl * T(d.elo[0]) + wxh * T(d.ehi[0]));
      sl.ey[m] = rb * (wyl * T(d.elo[1]) + wyh * T(d.ehi[1]));
      sl.qx[m] = rb * (wxl * T(d.qlo[0]) + wxh * T(d.qhi[0]));
      sl.qy[m] = rb * (wyl * T(d.qlo[1]) + wyh * T(d.qhi[1]));
      // second-order face terms on the diagonal (plain 1D centres, no Robin p)
      const T kxp = rx.k0 - sl.ex[m], kyp = ry.k0 - sl.ey[m];
      b1 = sl.qx[m] * kyp + sl.qy[m] * kxp;      // times mz0
      b2 = sl.qx[m] * ry.m0 + sl.qy[m] * rx.m0;  // times plain kz0
      b3 = kxp * ry.m0 + rx.m0 * kyp;            // times q_z at a z end
    } else {
      (void)wxl; (void)wxh; (void)wyl; (void)wyh; (void)rb;
    }
    const T kzp0 = T(16) * sl.zks, kzp1 = T(14) * sl.zks, kzp2 = T(7) * sl.zks, kzp3 = T(7) * sl.zks;
    sl.dv0[m] = T(1) / (a1 * mz0[0] + a2 * kz0[0] + b1 * mz0[0] + b2 * kzp0);
    sl.dv1[m] = T(1) / (a1 * mz0[1] + a2 * kz0[1] + b1 * mz0[1] + b2 * kzp1);
    sl.dv2[m] = T(1) / (a1 * mz0[2] + a2 * kz0[2] + b1 * mz0[2] + b2 * kzp2 + sl.zqlo * b3);
    sl.dv3[m] = T(1) / (a1 * mz0[3] + a2 * kz0[3] + b1 * mz0[3] + b2 * kzp3 + sl.zqhi * b3);
  }
}

template <typename T, int CPT, bool Q>
__device__ __forceinline__ T slot_dinv(const Slots<T, CPT, Q>& sl, int m, int k) {
  // blend with 0/1 weights: a select between struct fields would make the
  // compiler keep the whole slot state in scratch memory
  const int c = k + sl.zklo;
  const bool mid = (c & 1) != 0;
  const T w0 = mid ? T(1) : T(0);
  const T w2 = (!mid && c == 0) ? T(1) : T(0);
  const T w3 = (!mid && c == sl.zne2) ? T(1) : T(0);
  const T w1 = T(1) - w0 - w2 - w3;
  return w0 * sl.dv0[m] + w1 * sl.dv1[m] + w2 * sl.dv2[m] + w3 * sl.dv3[m];
}

template <typename T>
__device__ __forceinline__ void lds_zero(T* lds, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) lds[e] = T(0);
}

// The z-march, software-pipelined: fetch(li) issues the global loads of the
// operand at local index li = c + S k of the subdomain (always a valid node)
// kPrefetch planes ahead of its use; make(raw, li, own, dinv) turns them into
// the operand
// (own: the plane belongs to the slot's segment; dinv: inverse diagonal).
// store(li, en, i, j, k, q, p_k, dinv) receives the finished output at plane k
// of the slot's own segment, with the operand value p_k at that node (or the
// value make() carried for it), when en; make() and store() are called on every
// step and write nothing when own / en is false. Functors index pointers
// already offset to the subdomain (uniform base + 32-bit index).
constexpr int kPrefetch = 3;

// make() returns the operand of the stencil, or an operand with a separate
// value carried to store() (default: the operand itself).
template <typename T>
struct OpCarry {
  T op, carry;
};
template <typename T>
__device__ __forceinline__ T op_of(T v) { return v; }
template <typename T>
__device__ __forceinline__ T op_of(const OpCarry<T>& v) { return v.op; }
template <typename T>
__device__ __forceinline__ T carry_of(T v) { return v; }
template <typename T>
__device__ __forceinline__ T carry_of(const OpCarry<T>& v) { return v.carry; }

// ZU: the block marches one segment (G == 1), so every plane index is uniform
// across the block and the z-dependent row coefficients, the diagonal's
// z-kind and the plane tests run on the scalar unit.
template <bool ZU = false, typename T, int CPT, bool Q, class FetchF, class MakeF, class StoreF>
__device__ __forceinline__ void zmarch(const Slots<T, CPT, Q>& sl, T* lds, FetchF& fetch, MakeF& make,
                                       StoreF& store) {
  auto zlo = [&](int m) {
    if constexpr (ZU) return sl.uz0;
    else return sl.z0[m];
  };
  auto zhi = [&](int m) {
    if constexpr (ZU) return sl.uz1;
    else return sl.z1[m];
  };
  // coh: the plane lies outside the block's own z-range (another block of a
  // team writes it); edge: an own plane within two of the range's ends (the
  // neighbouring team members read it)
  auto coh_of = [&](int k) { return k < sl.uz0 || k >= sl.uz1; };
  // inverse diagonal at plane k; with uniform z the row kind is uniform and a
  // select chain on a scalar condition replaces the 0/1 blend
  auto dinv_of = [&](int m, int k) {
    if constexpr (ZU) {
      const int c = k + sl.zklo;
      const T d0 = sl.dv0[m], d1 = sl.dv1[m], d2 = sl.dv2[m], d3 = sl.dv3[m];
      T dv = (c & 1) != 0 ? d0 : d1;
      dv = c == 0 ? d2 : dv;
      dv = c == sl.zne2 ? d3 : dv;
      return dv;
    } else {
      return slot_dinv(sl, m, k);
    }
  };
  auto edge_of = [&](int k) { return k < sl.uz0 + 2 || k >= sl.uz1 - 2; };
  // operand loads of slot m at plane kq: fetch(li, coh), or fetch(li, coh, i,
  // j, kq) for a fetch that needs the node's local coordinates
  auto fetch_at = [&](int m, int kq) {
    const uint32_t li = uint32_t(sl.c[m] + sl.S * kq);
    if constexpr (std::is_invocable_v<FetchF&, uint32_t, bool, int, int, int>)
      return fetch(li, coh_of(kq), sl.i[m], sl.j[m], kq);
    else
      return fetch(li, coh_of(kq));
  };
  using Raw = decltype(fetch_at(0, 0));
  // operand of slot m at plane kc from its loads: make(raw, li, own, edge,
  // dinv), or with the node's local coordinates (i, j, kc) appended
  auto make_at = [&](const Raw& rv, int m, int kc, bool own) {
    const uint32_t li = uint32_t(sl.c[m] + sl.S * kc);
    if constexpr (std::is_invocable_v<MakeF&, Raw, uint32_t, bool, bool, T, int, int, int>)
      return make(rv, li, own, edge_of(kc), dinv_of(m, kc), sl.i[m], sl.j[m], kc);
    else
      return make(rv, li, own, edge_of(kc), dinv_of(m, kc));
  };
  // first operand plane of the march: two below the segment, or (uniform z)
  // the subdomain's first plane when the segment starts there, since planes
  // outside the subdomain contribute nothing
  // With uniform z the march also skips the halo plane that cannot reach an
  // own plane: a mid plane (odd closure index) couples only to its two
  // neighbouring planes, so below a mid first plane one halo plane suffices
  // (the plane under it is a mid plane too and reaches no own plane), and
  // likewise above a mid last plane. The skipped contributions are exact zeros.
  auto is_mid = [&](int k) { return ((k + sl.zklo) & 1) != 0; };
  auto kfirst = [&](int m) {
    if constexpr (ZU) return max(sl.uz0 - (is_mid(sl.uz0) ? 1 : 2), 0);
    else return sl.z0[m] - 2;
  };
  // last operand plane the march needs (uniform z); later steps only drain
  const int klast = ZU ? min(sl.uz1 - 1 + (is_mid(sl.uz1 - 1) ? 1 : 2), sl.nz - 1) : sl.nz - 1;
  T acc[CPT][5];
  T pr[CPT][3];
  // prefetch ring: slot q holds the operands of the step that is congruent to
  // q modulo kPrefetch. The step loop is unrolled kPrefetch times so every
  // slot is a fixed set of registers: a register receiving a load in flight is
  // never copied, so each use waits only for its own load.
  Raw raw[CPT][kPrefetch];
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[m][q] = T(0);
#pragma unroll
    for (int q = 0; q < 3; ++q) pr[m][q] = T(0);
#pragma unroll
    for (int q = 0; q < kPrefetch; ++q) {
      // unconditional load from a clamped, always valid plane: a fixed number
      // of loads per step lets every use wait for its own load only
      const int kq = min(max(kfirst(m) + q, 0), sl.nz - 1);
      raw[m][q] = fetch_at(m, kq);
    }
  }
  // the output of plane k is complete two steps after operand plane k + 2
  const int steps = ZU ? sl.uz1 + 2 - kfirst(0) : sl.seglen + 4;
  const int PX = sl.PX, SP = sl.SP;
  auto one_step = [&](auto ucst, int step) {
    constexpr int U = decltype(ucst)::value;
    // with second-order terms (the x-pass reads the operand plane) or
    // wave-owned rows (no barrier after the y-pass) the operand plane
    // alternates between two LDS planes, so the next step's writes never meet
    // this step's reads; otherwise the barrier after the y-pass orders them
    const int po = ((Q || sl.ra) && (step & 1)) ? 3 * SP : 0;
    bool inr[CPT];
    int kp[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      kp[m] = kfirst(m) + step;
      inr[m] = sl.act[m] && kp[m] >= 0 && kp[m] <= klast;
      // make() runs on every step (on a clamped, valid plane outside the
      // subdomain, with own = false): its stores are off, its result unused
      const int kc = min(max(kp[m], 0), sl.nz - 1);
      const bool own = sl.act[m] && kp[m] >= zlo(m) && kp[m] < zhi(m);
      const auto mv = make_at(raw[m][U], m, kc, own);
      if (inr[m]) lds[sl.lp[m] + po] = T(op_of(mv));
      // a plane outside the subdomain is never stored, so its carry is unused
      pr[m][2] = T(carry_of(mv));
      const int kq = min(max(kp[m] + kPrefetch, 0), sl.nz - 1);
      raw[m][U] = fetch_at(m, kq);
    }
    // uniform z: the steps past the last needed plane only drain the
    // accumulator ring and touch no LDS, so they skip both barriers
    const bool sync = !ZU || kfirst(0) + step <= klast;
    if (sync) __syncthreads();
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      if (inr[m]) {
        const T* P = lds + sl.lp[m] + po;
        const T a0 = P[0];
        const T s1 = P[-PX] + P[PX];
        const T s2 = P[-2 * PX] + P[2 * PX];
        const T u = sl.my0[m] * a0 + sl.my1 * s1 + sl.my2[m] * s2;
        const T v = sl.ky0[m] * a0 + sl.ky1 * s1 + sl.ky2[m] * s2;
        lds[sl.lp[m] + SP] = u;
        lds[sl.lp[m] + 2 * SP] = v;
      }
    }
    // wave-owned rows: the x-pass reads the y-pass results of its own wave
    // (LDS operations of a wave complete in order), and the next step's y-pass
    // rewrites them only after this wave's x-pass
    if (sync && !sl.ra) __syncthreads();
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      if (inr[m]) {
        const T* U_ = lds + sl.lp[m] + SP;
        const T* V = U_ + SP;
        const T u0 = U_[0], u1 = U_[-1] + U_[1], u2 = U_[-2] + U_[2];
        const T v0 = V[0], v1 = V[-1] + V[1], v2 = V[-2] + V[2];
        T Sx = sl.kx0[m] * u0 + sl.kx1 * u1 + sl.kx2[m] * u2 + sl.mx0[m] * v0 + sl.mx1 * v1 + sl.mx2[m] * v2;
        T Tx = sl.mx0[m] * u0 + sl.mx1 * u1 + sl.mx2[m] * u2;
        T zc = T(0);  // second-order z-face term of the centre row
        if constexpr (Q) if (sl.hasq) {
          // second-order faces q (tangential stiffness with plain 1D factors):
          // an x-face adds q (Ky (x) Mz + My (x) Kz) on its plane, a y-face
          // q (Kx (x) Mz + Mx (x) Kz), a z-face q (Kx (x) My + Mx (x) Ky)
          const T* P = lds + sl.lp[m] + po;
          const T p0 = P[0], p1 = P[-1] + P[1], p2 = P[-2] + P[2];
          const T pm = sl.mx0[m] * p0 + sl.mx1 * p1 + sl.mx2[m] * p2;
          const T pk = (sl.kx0[m] - sl.ex[m]) * p0 + sl.kx1 * p1 + sl.kx2[m] * p2;
          const T sf = sl.qx[m] * (v0 - sl.ey[m] * p0) + sl.qy[m] * pk;
          const T tf = sl.qx[m] * u0 + sl.qy[m] * pm;
          const int cz = kp[m] + sl.zklo;
          const T wzl = cz == 0 ? T(1) : T(0), wzh = cz == sl.zne2 ? T(1) : T(0);
          const T zq = wzl * sl.zqlo + wzh * sl.zqhi;
          const T ez = wzl * sl.zelo + wzh * sl.zehi;
          zc = zq * (Sx - sl.ex[m] * u0 - sl.ey[m] * pm) - ez * tf;
          Sx += sf;
          Tx += tf;
        }
        const Row<T> rz = row_of<T>(kp[m] + sl.zklo, sl.zne2, sl.zks, sl.zms, sl.zelo, sl.zehi);
        const T c1 = sl.mz1 * Sx + sl.kz1 * Tx;
        const T c2 = rz.m2 * Sx + rz.k2 * Tx;
        acc[m][0] += c2;
        acc[m][1] += c1;
        if constexpr (Q) acc[m][2] += rz.m0 * Sx + rz.k0 * Tx + zc;
        else acc[m][2] += rz.m0 * Sx + rz.k0 * Tx;
        acc[m][3] += c1;
        acc[m][4] = c2;
      } else {
        acc[m][4] = T(0);
      }
    }
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      {
        const int k = kp[m] - 2;
        const bool en = sl.act[m] && k >= zlo(m) && k < zhi(m);
        const int kc = min(max(k, 0), sl.nz - 1);
        store(uint32_t(sl.c[m] + sl.S * kc), en, edge_of(kc), sl.i[m], sl.j[m], kc, acc[m][0], pr[m][0],
              dinv_of(m, kc));
      }
      acc[m][0] = acc[m][1];
      acc[m][1] = acc[m][2];
      acc[m][2] = acc[m][3];
      acc[m][3] = acc[m][4];
      pr[m][0] = pr[m][1];
      pr[m][1] = pr[m][2];
    }
  };
  static_assert(kPrefetch == 3, "the step loop below is unrolled for a ring of three");
  int step = 0;
  for (; step + 3 <= steps; step += 3) {
    one_step(std::integral_constant<int, 0>(), step);
    one_step(std::integral_constant<int, 1>(), step + 1);
    one_step(std::integral_constant<int, 2>(), step + 2);
  }
  if (step < steps) one_step(std::integral_constant<int, 0>(), step++);
  if (step < steps) one_step(std::integral_constant<int, 1>(), step++);
}

template <typename T>
struct Pair {
  T a, b;
};

// Launch bound per x-y columns per thread (the host never launches more).
template <int CPT>
// Two columns per thread: up to 11 waves (3 per SIMD, 168 VGPRs); three: up to
// 8 waves (2 per SIMD, 256 VGPRs). A block a few waves larger than the plane
// needs spreads the second (third) column of the threads over more waves, so
// no SIMD carries more of them than the others.
struct Bound {
  static constexpr int value = CPT == 2 ? 704 : (CPT == 3 ? 512 : 1024);
};


// Robin data added to the local right-hand side at node (i, j, k).
struct LamOff {
  int64_t o[6];  // lambda offset per (local axis, side) face, -1 if none
  int32_t tswap; // SubDesc::tswap
};

__device__ __forceinline__ LamOff lam_offsets(const Dev& d, const SubDesc& sd) {
  LamOff L;
#pragma unroll
  for (int f = 0; f < 6; ++f) L.o[f] = sd.face[f] >= 0 ? d.faces[sd.face[f]].lam_off : -1;
  L.tswap = sd.tswap;
  return L;
}

// Node (t1, t2) of a face datum (t1 < t2 the local tangential axes, extents
// n1, n2): stored with the tangential axis of lower global index fastest.
__device__ __forceinline__ int64_t face_index(int t1, int t2, int n1, int n2, bool swap) {
  return swap ? t2 + (int64_t)n2 * t1 : t1 + (int64_t)n1 * t2;
}

__device__ __forceinline__ double lam_terms(const LamOff& L, const double* lam, int i, int j, int k, int nx,
                                            int ny, int nz) {
  double a = 0.0;
  const bool s0 = (L.tswap & 1) != 0, s1 = (L.tswap & 2) != 0, s2 = (L.tswap & 4) != 0;
  if (i == 0 && L.o[0] >= 0) a += lam[L.o[0] + face_index(j, k, ny, nz, s0)];
  if (i == nx - 1 && L.o[1] >= 0) a += lam[L.o[1] + face_index(j, k, ny, nz, s0)];
  if (j == 0 && L.o[2] >= 0) a += lam[L.o[2] + face_index(i, k, nx, nz, s1)];
  if (j == ny - 1 && L.o[3] >= 0) a += lam[L.o[3] + face_index(i, k, nx, nz, s1)];
  if (k == 0 && L.o[4] >= 0) a += lam[L.o[4] + face_index(i, j, nx, ny, s2)];
  if (k == nz - 1 && L.o[5] >= 0) a += lam[L.o[5] + face_index(i, j, nx, ny, s2)];
  return a;
}

// Algorithmic bytes of an inner solve of t CG iterations on subdomain sd:
// per iteration pass A reads r, p_old and writes p, q, pass B reads p, q, x, r
// and writes x, r (10 vectors; the first iteration reads neither p_old nor x),
// then the correction u += x reads x and u and writes u (FP64).
__device__ __forceinline__ unsigned long long cg_bytes(const SubDesc& sd, int t, int es) {
  if (t <= 0) return 0ull;
  const unsigned long long n = (unsigned long long)sd.n[0] * sd.n[1] * sd.n[2];
  return n * ((unsigned long long)(10 * t - 2) * es + es + 16ull);
}

// Algorithmic bytes of a fused inner solve of t >= 1 iterations: a
// preconditioned CG iteration with its dot products fused into the operator
// sweep moves 12 words per unknown (apply: read p, write q; updates of x, r, p
// and z = D^-1 r: 7; dots: 3), whatever the kernel keeps on chip; then
// u += x reads x and reads and writes u in FP64.
__device__ __forceinline__ unsigned long long fused_bytes(const SubDesc& sd, int t, int es) {
  if (t <= 0) return 0ull;
  const unsigned long long n = (unsigned long long)sd.n[0] * sd.n[1] * sd.n[2];
  return n * ((unsigned long long)(12 * t) * es + es + 16ull);
}

// ---------------------------------------------------------------------------- outer kernels

// Index of x-boundary node (i = 0 or n0 - 1, j, k) of subdomain sd in the
// x-boundary arrays (a subdomain one node thick along x uses the i = 0 half).
__device__ __forceinline__ int64_t xface_at(const SubDesc& sd, int i, int j, int k) {
  return sd.xoff + (i == 0 ? 0 : (int64_t)sd.n[1] * sd.n[2]) + j + (int64_t)sd.n[1] * k;
}

// Right-hand side at a boundary-shell node: bx (and fx = f, if given) on the
// x-boundary nodes, b elsewhere.
__device__ __forceinline__ void put_rhs(const SubDesc& sd, int i, int j, int64_t idx, int k, double fv, double v,
                                        double* __restrict__ b, double* __restrict__ fx, double* __restrict__ bx) {
  if (i == 0 || i == sd.n[0] - 1) {
    const int64_t xi = xface_at(sd, i, j, k);
    bx[xi] = v;
    if (fx) fx[xi] = fv;
  } else {
    b[idx] = v;
  }
}

// b = f + sum_j R_sj^T lambda_{s<-j} on the boundary-shell nodes of planes
// [z0, z1) of subdomain sd (off the shell b = f is left as it is), and fx = f
// there on the x-boundary nodes: the z-face planes whole, the other planes'
// perimeters; every node is written by the block that owns its plane.
__device__ __forceinline__ void shell_rhs(const Dev& d, const SubDesc& sd, int z0, int z1,
                                          const double* __restrict__ f, const double* __restrict__ lam,
                                          double* __restrict__ b, double* __restrict__ fx,
                                          double* __restrict__ bx) {
  const int nx = sd.n[0], ny = sd.n[1], nz = sd.n[2], S = nx * ny;
  const int xs = nx > 1 ? 2 : 1, ys = ny > 1 ? 2 : 1, ix = max(nx - 2, 0);
  const int perim = xs * ny + ys * ix;
  const int nzf = (z0 == 0 ? 1 : 0) + (z1 == nz && nz - 1 != 0 ? 1 : 0);  // z-face planes in range
  const int k0 = z0 == 0 ? 1 : z0, k1 = z1 == nz ? nz - 1 : z1;            // perimeter-only planes
  const int n_face = nzf * S, total = n_face + max(k1 - k0, 0) * perim;
  const LamOff L = lam_offsets(d, sd);
#pragma unroll 4
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int i, j, k;
    if (t < n_face) {
      k = (t < S && z0 == 0) ? 0 : nz - 1;
      const int e = t % S;
      i = e % nx;
      j = e / nx;
    } else {
      const int q = (t - n_face) / perim, e = (t - n_face) - q * perim;
      k = k0 + q;
      if (e < xs * ny) {
        i = e < ny ? 0 : nx - 1;
        j = e < ny ? e : e - ny;
      } else {
        const int e2 = e - xs * ny;
        j = e2 < ix ? 0 : ny - 1;
        i = 1 + (e2 < ix ? e2 : e2 - ix);
      }
    }
    const int64_t idx = sd.off + i + (int64_t)nx * (j + (int64_t)ny * k);
    const double fv = f[idx];
    put_rhs(sd, i, j, idx, k, fv, fv + lam_terms(L, lam, i, j, k, nx, ny, nz), b, fx, bx);
  }
}

// b = f + sum_j R_sj^T lambda_{s<-j} on the nodes of planes [z0, z1) of
// subdomain sd that lie on two or more planes of the box's boundary (edges and
// corners; every node of a plane when the subdomain is one node thick along x
// or y, of a z-face plane when it is one node thick along z). The exchange
// writes b at the nodes of one face; only these need the sum of several.
__device__ __forceinline__ void shell_edges(const Dev& d, const SubDesc& sd, int z0, int z1,
                                            const double* __restrict__ f, const double* __restrict__ lam,
                                            double* __restrict__ b, double* __restrict__ bx) {
  const int nx = sd.n[0], ny = sd.n[1], nz = sd.n[2], S = nx * ny;
  const bool thin = nx == 1 || ny == 1;
  // per plane: a z-face plane has its perimeter (or all of it), another plane
  // its four corner columns (or all of it)
  const int perim = (thin || nz == 1) ? S : 2 * nx + 2 * (ny - 2);
  const int inner = thin ? S : 4;
  const bool lo = z0 == 0, hi = z1 == nz && nz > 1;
  const int nzf = (lo ? 1 : 0) + (hi ? 1 : 0);
  const int k0 = lo ? 1 : z0, k1 = hi ? nz - 1 : z1;
  const int n_face = nzf * perim, total = n_face + max(k1 - k0, 0) * inner;
  const LamOff L = lam_offsets(d, sd);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int i, j, k, e;
    bool whole;
    if (t < n_face) {
      k = (t < perim && lo) ? 0 : nz - 1;
      e = t < perim ? t : t - perim;
      whole = perim == S;
    } else {
      const int q = (t - n_face) / inner;
      k = k0 + q;
      e = (t - n_face) - q * inner;
      whole = thin;
      if (!whole) {  // corner columns
        i = (e & 1) ? nx - 1 : 0;
        j = (e & 2) ? ny - 1 : 0;
      }
    }
    if (whole) {
      i = e % nx;
      j = e / nx;
    } else if (t < n_face) {  // perimeter of a z-face plane (nx, ny >= 2)
      if (e < 2 * ny) {
        i = e < ny ? 0 : nx - 1;
        j = e < ny ? e : e - ny;
      } else {
        const int e2 = e - 2 * ny, ix = nx - 2;
        j = e2 < ix ? 0 : ny - 1;
        i = 1 + (e2 < ix ? e2 : e2 - ix);
      }
    }
    const int64_t idx = sd.off + i + (int64_t)nx * (j + (int64_t)ny * k);
    put_rhs(sd, i, j, idx, k, 0.0, f[idx] + lam_terms(L, lam, i, j, k, nx, ny, nz), b, nullptr, bx);
  }
}

// r = b - A u with b = f + sum_j R_sj^T lambda_{s<-j}. b holds f inside the
// subdomain, f + lambda on the nodes of one face (written by the exchange, or
// by k_shell_rhs at the start of a run); each block first rewrites the edge
// and corner nodes of its own planes, where several faces' data add. On the
// x-boundary nodes (i = 0, n0 - 1) the right-hand side lives in bx instead, a
// contiguous array per subdomain face (in b those nodes are one cache line
// apart, too costly for the exchange to write). RZ: also r'D^-1 r (the
// stepwise CG's first gamma). ZU: every block marches one segment (the host
// checks; otherwise the partials are NaN and the solve reports a breakdown).
template <typename TO, int CPT, bool Q, bool RZ, bool ZU = false>
__global__ void __launch_bounds__(Bound<CPT>::value) k_residual(Dev d, const BlockDesc* blocks, const double* __restrict__ u,
                                                   const double* __restrict__ f, const double* __restrict__ lam,
                                                   double* __restrict__ b, double* __restrict__ bx,
                                                   TO* __restrict__ r, double* __restrict__ part,
                                                   double* __restrict__ team_part) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* lds = reinterpret_cast<double*>(smem);
  // the fused kernel that follows tags its team partials from epoch 0: clear
  // every slot (tag 0)
  if (team_part && blockIdx.x == 0)
    for (int i = threadIdx.x; i < d.geo.n_sub * kMaxTeam * 2 * 4; i += blockDim.x) team_part[i] = 0.0;
  const BlockDesc bd = blocks[blockIdx.x];
  const SubDesc sd = d.subs[bd.s];
  shell_edges(d, sd, bd.z0, bd.z1, f, lam, b, bx);
  Slots<double, CPT, Q> sl;
  slots_init(sl, sd, d.geo, bd.z0, bd.z1, true);
  lds_zero(lds, sl.G * kPlanes * sl.SP);
  // the block's b writes are visible to its own march after the barrier
  __syncthreads();
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const bool bad = ZU && sl.G != 1;
  const double* __restrict__ ub = u + sl.off;
  const double* __restrict__ bb = b + sl.off;
  TO* __restrict__ rb = r + sl.off;
  // u is prefetched with the operand ring; b is loaded when its plane's
  // operand is made and carried to the store two steps later (were it part
  // of the ring, its register would stay live after its reload is issued and
  // the register allocator would copy every reloaded entry at the loop's end,
  // waiting for all loads in flight)
  auto fetch = [=](uint32_t li, bool) { return at(ub, li); };
  // the right-hand side of an x-boundary column comes from bx (one address
  // select per node, one load either way)
  const int nx1 = sd.n[0] - 1, ny = sd.n[1];
  const int64_t nynz = (int64_t)sd.n[1] * sd.n[2];
  const double* __restrict__ xb = bx + sd.xoff;
  auto make = [=](double v, uint32_t li, bool, bool, double, int i, int j, int k) {
    const double* p = (i == 0 || i == nx1) ? xb + ((i == 0 ? 0 : nynz) + j + (int64_t)ny * k) : bb + li;
    return OpCarry<double>{v, *p};
  };
  auto store = [&](uint32_t li, bool en, bool, int, int, int, double q, double bv, double dinv) {
    if (!en) return;
    const TO rt = TO(bv - q);
    at(rb, li) = rt;
    const double rd = double(rt);
    if constexpr (RZ) a0 += rd * rd * dinv;
    else (void)dinv;
    a1 += rd * rd;
    a2 += bv * bv;
  };
  if (!bad) zmarch<ZU>(sl, lds, fetch, make, store);
  double acc[3] = {a0, a1, a2};
  block_sum(acc);
  if (bad) acc[0] = acc[1] = acc[2] = __builtin_nan("");
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = acc[0];
    part[3 * blockIdx.x + 1] = acc[1];
    part[3 * blockIdx.x + 2] = acc[2];
  }
}

// y = A x (diagnostic).
template <typename T, int CPT, bool Q>
__global__ void __launch_bounds__(Bound<CPT>::value) k_apply(Dev d, const BlockDesc* blocks, const T* __restrict__ x,
                                                T* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const BlockDesc bd = blocks[blockIdx.x];
  const SubDesc sd = d.subs[bd.s];
  Slots<T, CPT, Q> sl;
  slots_init(sl, sd, d.geo, bd.z0, bd.z1, true);
  lds_zero(lds, sl.G * kPlanes * sl.SP);
  __syncthreads();
  const T* __restrict__ xb = x + sl.off;
  T* __restrict__ yb = y + sl.off;
  auto fetch = [=](uint32_t li, bool) { return at(xb, li); };
  auto make = [](T v, uint32_t, bool, bool, T) { return v; };
  auto store = [=](uint32_t li, bool en, bool, int, int, int, T q, T, T) {
    if (en) at(yb, li) = q;
  };
  zmarch(sl, lds, fetch, make, store);
}

// Pass B of a CG iteration over the slot's planes [z0, z1): x += alpha p,
// r -= alpha q, accumulating r'D^-1 r and r'r. Four planes per round so that
// sixteen loads are in flight before the first use.
template <typename T, int CPT, bool Q>
__device__ __forceinline__ void cg_pass_b(const Slots<T, CPT, Q>& sl, bool first, T alpha, T* __restrict__ x,
                                          const T* __restrict__ p, T* __restrict__ r, const T* __restrict__ q,
                                          double& arz, double& arr) {
  T* __restrict__ xb = x + sl.off;
  const T* __restrict__ pb = p + sl.off;
  T* __restrict__ rb = r + sl.off;
  const T* __restrict__ qb = q + sl.off;
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
    if (!sl.act[m]) continue;
    for (int k = sl.z0[m]; k < sl.z1[m]; k += 4) {
      T pv[4], xv[4], rv[4], qv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k + u;
        if (kk < sl.z1[m]) {
          const uint32_t li = sl.c[m] + sl.S * kk;
          pv[u] = at(pb, li);
          xv[u] = first ? T(0) : at(xb, li);
          rv[u] = at(rb, li);
          qv[u] = at(qb, li);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k + u;
        if (kk < sl.z1[m]) {
          const uint32_t li = sl.c[m] + sl.S * kk;
          at(xb, li) = xv[u] + alpha * pv[u];
          const T rn = rv[u] - alpha * qv[u];
          at(rb, li) = rn;
          const double rd = double(rn);
          arz += rd * rd * double(slot_dinv(sl, m, kk));
          arr += rd * rd;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------- stepwise CG


template <typename T, int CPT, bool Q, bool ZU = false>
__global__ void __launch_bounds__(Bound<CPT>::value) k_cg_apply(Dev d, const BlockDesc* blocks, const int32_t* __restrict__ bfirst,
                                                   int t, int max_inner, const T* __restrict__ r,
                                                   const T* __restrict__ pold, T* __restrict__ pnew,
                                                   T* __restrict__ q, double* __restrict__ part,
                                                   CgScal* __restrict__ scal, int32_t* ndone,
                                                   unsigned long long* counters, int32_t* flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const BlockDesc bd = blocks[blockIdx.x];
  const int s = bd.s;
  if (scal[s].done) return;
  const int b0 = bfirst[s], b1 = bfirst[s + 1];
  const bool leader = ((int)blockIdx.x == b0) && (threadIdx.x == 0);
  double rz, rr;
  if (t == 0) {
    rz = scal[s].rz[0];
    rr = scal[s].rr0;
  } else {
    rz = 0.0;
    rr = 0.0;
    for (int b = b0; b < b1; ++b) {
      rz += part[3 * b + 1];
      rr += part[3 * b + 2];
    }
  }
  const bool bad = !isfinite(rr) || !isfinite(rz);
  if (bad || !(rr > scal[s].stop2) || t >= max_inner) {
    if (leader) {
      scal[s].done = 1;
      scal[s].iters = t;
      scal[s].breakdown = bad ? kBrkNonFinite : 0;
      if (bad) atomicOr(flags, kBrkNonFinite);
      atomicAdd(ndone, 1);
      const SubDesc& sd = d.subs[s];
      atomicAdd(&counters[0], (unsigned long long)t);
      atomicAdd(&counters[1], cg_bytes(sd, t, sizeof(T)));
    }
    return;
  }
  const double beta = t == 0 ? 0.0 : rz / scal[s].rz[(t - 1) & 1];
  if (leader) scal[s].rz[t & 1] = rz;
  const SubDesc sd = d.subs[s];
  Slots<T, CPT, Q> sl;
  slots_init(sl, sd, d.geo, bd.z0, bd.z1, true);
  lds_zero(lds, sl.G * kPlanes * sl.SP);
  __syncthreads();
  const T tb = T(beta);
  const bool first = t == 0;
  double a0 = 0.0;
  const T* __restrict__ rb = r + sl.off;
  const T* __restrict__ pob = pold + sl.off;
  T* __restrict__ pnb = pnew + sl.off;
  T* __restrict__ qb = q + sl.off;
  auto fetch = [=](uint32_t li, bool) { return Pair<T>{at(rb, li), at(pob, li)}; };
  auto make = [=](Pair<T> v, uint32_t li, bool own, bool, T dinv) {
    const T pn = dinv * v.a + (first ? T(0) : tb * v.b);
    if (own) at(pnb, li) = pn;
    return pn;
  };
  auto store = [&](uint32_t li, bool en, bool, int, int, int, T qv, T pk, T) {
    if (!en) return;
    at(qb, li) = qv;
    a0 += double(pk) * double(qv);
  };
  // ZU: the host launches it only when every block marches one segment;
  // otherwise the NaN partial ends the solve with a breakdown
  const bool badseg = ZU && sl.G != 1;
  if (!badseg) zmarch<ZU>(sl, lds, fetch, make, store);
  double acc[1] = {a0};
  block_sum(acc);
  if (badseg) acc[0] = __builtin_nan("");
  if (threadIdx.x == 0) part[3 * blockIdx.x] = acc[0];
}

template <typename T, int CPT, bool Q>
__global__ void __launch_bounds__(Bound<CPT>::value) k_cg_update(Dev d, const BlockDesc* blocks, const int32_t* __restrict__ bfirst,
                                                    int t, T* __restrict__ x, const T* __restrict__ p,
                                                    T* __restrict__ r, const T* __restrict__ q,
                                                    double* __restrict__ part, CgScal* __restrict__ scal,
                                                    int32_t* ndone, int32_t* flags) {
  const BlockDesc bd = blocks[blockIdx.x];
  const int s = bd.s;
  if (scal[s].done) return;
  const int b0 = bfirst[s], b1 = bfirst[s + 1];
  double pq = 0.0;
  for (int b = b0; b < b1; ++b) pq += part[3 * b];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if ((int)blockIdx.x == b0 && threadIdx.x == 0) {
      const int32_t why = isfinite(pq) ? kBrkCurvature : kBrkNonFinite;
      scal[s].done = 1;
      scal[s].iters = t;
      scal[s].breakdown = why;
      atomicOr(flags, why);
      atomicAdd(ndone, 1);
    }
    return;
  }
  const T alpha = T(scal[s].rz[t & 1] / pq);
  const SubDesc sd = d.subs[s];
  Slots<T, CPT, Q> sl;
  slots_init(sl, sd, d.geo, bd.z0, bd.z1, true);
  double a0 = 0.0, a1 = 0.0;
  cg_pass_b(sl, t == 0, alpha, x, p, r, q, a0, a1);
  double acc[2] = {a0, a1};
  block_sum(acc);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 1] = acc[0];
    part[3 * blockIdx.x + 2] = acc[1];
  }
}

template <typename T, int CPT>
__global__ void __launch_bounds__(Bound<CPT>::value) k_add_correction(Dev d, const BlockDesc* blocks, double* __restrict__ u,
                                                         const T* __restrict__ x, const CgScal* __restrict__ scal) {
  const BlockDesc bd = blocks[blockIdx.x];
  if (scal[bd.s].iters <= 0 || scal[bd.s].breakdown) return;
  const SubDesc sd = d.subs[bd.s];
  Slots<T, CPT, false> sl;
  slots_init(sl, sd, d.geo, bd.z0, bd.z1, true);
  double* __restrict__ ub = u + sl.off;
  const T* __restrict__ xb = x + sl.off;
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
    if (!sl.act[m]) continue;
    for (int k = sl.z0[m]; k < sl.z1[m]; ++k) {
      const uint32_t li = sl.c[m] + sl.S * k;
      at(ub, li) += double(at(xb, li));
    }
  }
}

// ---------------------------------------------------------------------------- fused CG

template <typename T>
struct Five {
  T r, w, s, p, x;
};
template <typename T>
struct Three {
  T r, w, s;
};
template <typename T>
struct Four {
  T r, w, s, p;
};

// Sum the block partials of the T members of a team (the blocks that share
// one subdomain). Every store of the block's sweep completes first (the halo
// planes the other members read next were written with coherent stores);
// then the block publishes its partials with coherent stores, each carrying
// the epoch in its eight lowest mantissa bits, and lanes of the first wave
// spin (bounded) on the T members' slots until every tag reads the epoch:
// arrival and data in one round trip. The tag costs at most 2^-44 of a
// partial's value; the tagged bits are cleared and the partials summed in
// member order, so every member gets the same sums. Epoch e uses slots
// (e & 1) with tag (e + 1) mod 256; the slots are zeroed (tag 0) before each
// launch, and a slot's previous tag is that of epoch e - 2, never equal.
// A member that waits longer than a.spin_ticks (wall clock, 100 MHz; the host
// default is 2^27 ticks, about 1.3 s) for the others gives up and reports a
// failed barrier (kBrkBarrier): the wait always ends.
//
// Why no cache write-back or invalidation is needed. On gfx950 the L2 cache
// belongs to one XCD and is not coherent with the other XCDs' L2 caches. Every
// value one member writes and another reads -- the halo planes of r, w, s and
// the tagged partials -- is written and read only with agent-scope atomic
// stores and loads (st_coh / ld_coh). Those carry the sc1 cache policy: a
// store is written through to memory that every XCD sees, and a load does not
// hit a stale line in its own XCD's L2. Ordering: (1) every wave waits for all
// of its vector memory operations to complete (s_waitcnt vmcnt(0): stores
// complete only once written through) and then the workgroup barrier, so all
// halo stores of the block are visible device-wide before thread 0 stores the
// tagged partials; (2) a reader sees a partial's tag only after that store,
// hence after every halo store of that member; (3) the waves of the reader
// load the next sweep's halo planes only after the workgroup barrier that
// follows the tag check (the march issues its first prefetch after the
// barrier; loads left over from the previous march are never used). This is
// the AMDGPU memory model's implementation of an agent-scope release and
// acquire restricted to atomic accesses; the L2 write-back and invalidation
// that a general release/acquire adds only serve non-atomic accesses, and the
// members never share data through those (p and x stay with their owner).
constexpr int kTeamSlot = 4;  // doubles per (member, parity) slot

__device__ __forceinline__ double with_tag(double v, unsigned tag) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return __longlong_as_double((long long)((b & ~0xFFull) | tag));
}
__device__ __forceinline__ unsigned tag_of(double v) {
  return (unsigned)((unsigned long long)__double_as_longlong(v) & 0xFFull);
}

template <int N>
__device__ __forceinline__ void team_sum(double (&v)[N], const FusedArgs& a, int s, int tau, int TM, int epoch,
                                         int& fail) {
  static_assert(N <= kTeamSlot, "partials per slot");
  if (TM <= 1) return;
  __shared__ double tval[kMaxTeam * N];
  __shared__ int tfl[kMaxTeam * N];
  const unsigned tag = (unsigned)((epoch + 1) & 0xFF);
  const unsigned want = (unsigned)((epoch + 1 + a.tag_skew) & 0xFF);
  double* const base = a.team_part + (size_t)s * kMaxTeam * 2 * kTeamSlot;
  wait_vm_all();
  __syncthreads();
  if (threadIdx.x == 0) {
    double* slot = base + ((size_t)tau * 2 + (epoch & 1)) * kTeamSlot;
#pragma unroll
    for (int n = 0; n < N; ++n) st_coh(&slot[n], with_tag(v[n], tag));
  }
  if ((int)threadIdx.x < TM * N) {
    const int m = threadIdx.x / N, n = threadIdx.x - m * N;
    const double* q = base + ((size_t)m * 2 + (epoch & 1)) * kTeamSlot + n;
    double val = ld_coh(q);
    const unsigned long long t0 = wall_clock64();
    int f = 0;
    while (tag_of(val) != want) {
      if (wall_clock64() - t0 > a.spin_ticks) {
        f = 1;
        break;
      }
      val = ld_coh(q);
    }
    tval[threadIdx.x] = with_tag(val, 0u);
    tfl[threadIdx.x] = f;
  }
  __syncthreads();
  int f = 0;
#pragma unroll
  for (int n = 0; n < N; ++n) {
    double acc = 0.0;
    for (int m = 0; m < TM; ++m) {
      acc += tval[m * N + n];
      f |= tfl[m * N + n];
    }
    v[n] = acc;
  }
  fail |= f;
  // tval is rewritten only after the next sweep's barriers
}

// One block per subdomain (team = 1), or a team of blocks each owning a
// contiguous range of z-planes (team > 1): the complete preconditioned CG solve of
// A_s d = r_s from d = 0, then u_s += d. No inter-block communication.
// The CG is the single-reduction form of Chronopoulos and Gear: with
// u = D^-1 r and w = A u carried along, one sweep per iteration updates
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = D^-1 r
// pointwise and applies w = A u, and one block reduction yields
// gamma = r'u, delta = w'u and r'r; then beta = gamma/gamma_old and
// alpha = gamma / (delta - beta gamma / alpha_old). r, w, s, p are double
// buffered (halo planes of one segment are read while another writes).
// COH (a team of more than one block): every load and store of the vectors
// whose halo planes the team members read is coherent (ld_coh / st_coh), so
// the team barrier needs no cache maintenance; a fixed instruction form on
// every plane keeps the prefetch waits exact.
// RES (uniform z only): 1, p and x stay in LDS for the whole launch; 2, x
// alone (for z-ranges where both do not fit). A halo plane only needs
// u = D^-1 (r - alpha (w + beta s)), so p and x are read and written by the
// thread that owns the node and never by another block; global traffic per CG
// iteration drops from ten words per node to six (eight with x alone).
template <typename T, int CPT, bool Q, bool ZU, bool COH, int RES>
__global__ void __launch_bounds__(Bound<CPT>::value) k_fused_cg(Dev d, const int32_t* __restrict__ bfirst, FusedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  // block -> (subdomain s, member tau of its team of TM blocks), host-built:
  // the members of a team share blockIdx % 8, i.e. one XCD (shared L2)
  const TeamSlot ts = a.fmap[blockIdx.x];
  if (ts.s < 0) return;  // padding
  const int s = ts.s, tau = ts.tau, TM = ts.T;
  const SubDesc sd = d.subs[s];
  const int zb0 = (tau * sd.n[2]) / TM, zb1 = ((tau + 1) * sd.n[2]) / TM;
  Slots<T, CPT, Q> sl;
  const bool ra = a.rows != 0;
  slots_init(sl, sd, d.geo, zb0, zb1, true, ra);
  int epoch = 0, tfail = 0;
  // buffers chosen with selects, never through an indexed array: pointers
  // read back from a private array lose their global address space and the
  // loads become flat loads, which every barrier then waits for
  T* const r0b = reinterpret_cast<T*>(a.r);
  T* const r1b = reinterpret_cast<T*>(a.r1);
  T* const w0b = reinterpret_cast<T*>(a.w0);
  T* const w1b = reinterpret_cast<T*>(a.w1);
  T* const s0b = reinterpret_cast<T*>(a.s0);
  T* const s1b = reinterpret_cast<T*>(a.s1);
  T* const p0b = reinterpret_cast<T*>(a.p0);
  T* const p1b = reinterpret_cast<T*>(a.p1);
  T* __restrict__ x = reinterpret_cast<T*>(a.x);
  double rr = 0.0, bb = 0.0;
  for (int b = bfirst[s]; b < bfirst[s + 1]; ++b) {
    rr += a.res_part[3 * b + 1];
    bb += a.res_part[3 * b + 2];
  }
  const double stop2 = fmax(a.tol_rel * a.tol_rel * rr, a.tol_abs * a.tol_abs * bb);
  // The inner solve runs on sig r instead of r, sig a power of two that brings
  // the mean square of r near one: exact scaling, undone when x is added to u.
  // Without it the outer iteration's convergence drives r towards 1e-22 and the
  // FP32 products of the dot products into the subnormal range.
  int sexp = 0;
  if (isfinite(rr) && rr > 0.0) {
    int e2 = 0;
    (void)frexp(rr / double(sd.n[0] * sd.n[1] * sd.n[2]), &e2);
    sexp = min(max(-(e2 / 2), -100), 100);
  }
  const T tsig = T(ldexp(1.0, sexp));
  const double isig = ldexp(1.0, -sexp);
  const double stop2s = stop2 * ldexp(1.0, 2 * sexp);
  // march planes: the second operand plane only with second-order terms or
  // wave-owned rows (see zmarch)
  const int mplanes = RES ? march_planes(Q, ra) : kPlanes;
  // march planes, and the resident x (and p) of the first CG iteration where
  // the launch's LDS holds them (else the block reports a launch mismatch)
  const int res_words = (RES && ZU) ? (RES == 1 ? 2 : 1) * (zb1 - zb0) * sl.S : 0;
  const bool res_fit = (size_t)(sl.G * mplanes * sl.SP + res_words) * sizeof(T) <= a.lds_bytes;
  lds_zero(lds, sl.G * mplanes * sl.SP + (res_fit ? res_words : 0));
  __syncthreads();
  // resident p (RES 1) and x: one LDS value per own node, index li - S uz0
  T* const xres = lds + sl.G * mplanes * sl.SP;
  T* const pres = xres + (size_t)(zb1 - zb0) * sl.S;
  const uint32_t plane0 = (uint32_t)(sl.S * zb0);
  int t = 0, brk = 0;  // brk: BreakBits of this block
  if (RES && (!ZU || !res_fit)) brk |= kBrkLaunch;  // the host sizes the LDS for the largest z-range
  if (!COH && TM > 1) brk |= kBrkLaunch;  // the host picks the coherent variant whenever a team has 2+ blocks
  if (!isfinite(rr) || !isfinite(bb)) brk |= kBrkNonFinite;
  if (ZU && sl.G != 1) brk |= kBrkLaunch;  // the host selects ZU only when every block has one segment
  // wave-owned rows only where the block's waves cover the plane (host checked)
  if (ra && (!ZU || ra_waves(sd.n[0], sd.n[1], CPT) < 1 || ra_waves(sd.n[0], sd.n[1], CPT) > (int)(blockDim.x >> 6)))
    brk |= kBrkLaunch;
  if (!brk && rr > stop2 && a.max_inner > 0) {
    // u0 = D^-1 r0, w0 = A u0, gamma0 = r0'u0, delta0 = w0'u0
    double g0 = 0.0, d0 = 0.0;
    {
      const T* __restrict__ r0 = r0b + sl.off;
      T* __restrict__ w0 = w0b + sl.off;
      auto fetch = [=](uint32_t li, bool) { return at(r0, li); };  // r0: written by an earlier launch
      auto make = [&](T rv0, uint32_t, bool own, bool, T dinv) {
        const T rv = rv0 * tsig;
        const T u = dinv * rv;
        if (own) g0 += double(rv) * double(u);
        return u;
      };
      auto store = [&](uint32_t li, bool en, bool, int, int, int, T wv, T uk, T) {
        if (!en) return;
        if constexpr (COH) st_coh(&at(w0, li), wv);
        else at(w0, li) = wv;
        d0 += double(wv) * double(uk);
      };
      zmarch<ZU>(sl, lds, fetch, make, store);
    }
    double acc0[2] = {g0, d0};
    block_sum(acc0);
    team_sum(acc0, a, s, tau, TM, epoch++, tfail);
    double gamma = acc0[0], delta = acc0[1];
    double alpha = gamma / delta, beta = 0.0;
    if (tfail) brk |= kBrkBarrier;
    else if (!isfinite(gamma) || !isfinite(delta)) brk |= kBrkNonFinite;
    else if (!(delta > 0.0)) brk |= kBrkCurvature;
    while (!brk) {
      const bool odd = (t & 1) != 0;
      const T* __restrict__ rc = (odd ? r1b : r0b) + sl.off;
      const T* __restrict__ wc = (odd ? w1b : w0b) + sl.off;
      const T* __restrict__ sc = (odd ? s1b : s0b) + sl.off;
      const T* __restrict__ pc = (odd ? p1b : p0b) + sl.off;
      T* __restrict__ xs = x + sl.off;
      T* __restrict__ rn_ = (odd ? r0b : r1b) + sl.off;
      T* __restrict__ wn_ = (odd ? w0b : w1b) + sl.off;
      T* __restrict__ sn_ = (odd ? s0b : s1b) + sl.off;
      T* __restrict__ pn_ = (odd ? p0b : p1b) + sl.off;
      const bool first = t == 0;
      const T ta = T(alpha), tb = T(beta), rsc = first ? tsig : T(1);
      // per-thread partial sums in the inner precision (a few dozen terms),
      // combined across the block in FP64
      T ag = T(0), ad = T(0), ar = T(0);
      auto fetch = [=](uint32_t li, bool) {
        if constexpr (RES == 2) {
          Four<T> v;
          if constexpr (COH) {
            v.r = ld_coh(&at(rc, li));
            v.w = ld_coh(&at(wc, li));
            v.s = ld_coh(&at(sc, li));
          } else {
            v.r = at(rc, li);
            v.w = at(wc, li);
            v.s = at(sc, li);
          }
          v.p = at(pc, li);  // p: own planes only, never exchanged
          return v;
        } else if constexpr (RES == 1) {
          Three<T> v;
          if constexpr (COH) {
            v.r = ld_coh(&at(rc, li));
            v.w = ld_coh(&at(wc, li));
            v.s = ld_coh(&at(sc, li));
          } else {
            v.r = at(rc, li);
            v.w = at(wc, li);
            v.s = at(sc, li);
          }
          return v;
        } else {
        Five<T> v;
        if constexpr (COH) {
          v.r = ld_coh(&at(rc, li));
          v.w = ld_coh(&at(wc, li));
          v.s = ld_coh(&at(sc, li));
          v.p = ld_coh(&at(pc, li));
        } else {
          v.r = at(rc, li);
          v.w = at(wc, li);
          v.s = at(sc, li);
          v.p = at(pc, li);
        }
        v.x = at(xs, li);  // x: own planes only, never exchanged
        return v;
        }
      };
      auto make = [&](const auto& v, uint32_t li, bool own, bool, T dinv) {
        // the first iteration has no previous direction: beta = 0 there, and
        // the direction buffers hold finite values (cleared before every run
        // of outer iterations, finite after every launch that does not end
        // the solve), so beta s and beta p vanish without a select; the
        // resident x (and p) start at zero
        const T vr = v.r * rsc;  // r0 comes unscaled from the residual kernel
        const T sn = v.w + tb * v.s;
        const T rn = vr - ta * sn;
        const T un = dinv * rn;
        if constexpr (RES != 0) {
          if (own) {
            const uint32_t q = li - plane0;
            T pn;
            if constexpr (RES == 1) {
              pn = fma(tb, pres[q], dinv * vr);
              pres[q] = pn;
            } else {
              pn = fma(tb, v.p, dinv * vr);
              at(pn_, li) = pn;
            }
            xres[q] = fma(ta, pn, xres[q]);
            if constexpr (COH) {
              st_coh(&at(sn_, li), sn);
              st_coh(&at(rn_, li), rn);
            } else {
              at(sn_, li) = sn;
              at(rn_, li) = rn;
            }
            ag += rn * un;
            ar += rn * rn;
          }
          return un;
        } else {
        // the same rounding as the resident form: explicit fused multiply-adds
        // (the global x still holds the last outer iteration's correction)
        const T vx = first ? T(0) : v.x;
        const T pn = fma(tb, v.p, dinv * vr);
        if (own) {
          if constexpr (COH) {
            st_coh(&at(pn_, li), pn);
            st_coh(&at(sn_, li), sn);
            st_coh(&at(rn_, li), rn);
          } else {
            at(pn_, li) = pn;
            at(sn_, li) = sn;
            at(rn_, li) = rn;
          }
          at(xs, li) = fma(ta, pn, vx);
          ag += rn * un;
          ar += rn * rn;
        }
        return un;
        }
      };
      auto store = [&](uint32_t li, bool en, bool, int, int, int, T wv, T uk, T) {
        if (!en) return;
        if constexpr (COH) st_coh(&at(wn_, li), wv);
        else at(wn_, li) = wv;
        ad += wv * uk;
      };
      zmarch<ZU>(sl, lds, fetch, make, store);
      double acc[3] = {double(ag), double(ad), double(ar)};
      block_sum(acc);
      team_sum(acc, a, s, tau, TM, epoch++, tfail);
      ++t;
      rr = acc[2];
      if (tfail) {
        brk |= kBrkBarrier;
        break;
      }
      if (!isfinite(acc[0]) || !isfinite(acc[1]) || !isfinite(rr)) {
        brk |= kBrkNonFinite;
        break;
      }
      if (!(rr > stop2s) || t >= a.max_inner) break;
      const double gnew = acc[0];
      beta = gnew / gamma;
      const double den = acc[1] - beta * gnew / alpha;
      if (!(den > 0.0)) {
        brk |= isfinite(den) ? kBrkCurvature : kBrkNonFinite;
        break;
      }
      alpha = gnew / den;
      gamma = gnew;
    }
  }
  // a subdomain whose solve broke down keeps its iterate (the host reports it)
  if (t > 0 && !brk) {
    const T* __restrict__ xb = x + sl.off;
    double* __restrict__ ub = a.u + sl.off;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      if (!sl.act[m]) continue;
      for (int k = sl.z0[m]; k < sl.z1[m]; k += 4) {
        T xv[4];
        double uv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (k + u < sl.z1[m]) {
            const uint32_t li = sl.c[m] + sl.S * (k + u);
            xv[u] = RES != 0 ? xres[li - plane0] : at(xb, li);
            uv[u] = at(ub, li);
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (k + u < sl.z1[m]) at(ub, sl.c[m] + sl.S * (k + u)) = uv[u] + double(xv[u]) * isig;
      }
    }
  }
  if (threadIdx.x == 0 && brk) atomicOr(a.flags, brk);
  if (threadIdx.x == 0 && tau == 0) {
    a.scal[s].iters = t;
    a.scal[s].breakdown = brk;
    a.scal[s].done = 1;
    atomicAdd(&a.iters_total[0], (unsigned long long)t);
    atomicAdd(&a.iters_total[1], fused_bytes(sd, t, sizeof(T)));
  }
}

#define SOS_DISPATCH_Q(hasq, CALL) \
  if (hasq) {                       \
    constexpr bool Q = true;        \
    CALL;                           \
  } else {                          \
    constexpr bool Q = false;       \
    CALL;                           \
  }

#define SOS_DISPATCH_CPT(cpt, KERNEL_CALL) \
  switch (cpt) {                           \
    case 1: {                              \
      constexpr int C = 1;                 \
      KERNEL_CALL;                         \
    } break;                               \
    case 2: {                              \
      constexpr int C = 2;                 \
      KERNEL_CALL;                         \
    } break;                               \
    case 3: {                              \
      constexpr int C = 3;                 \
      KERNEL_CALL;                         \
    } break;                               \
    case 4: {                              \
      constexpr int C = 4;                 \
      KERNEL_CALL;                         \
    } break;                               \
    default:                               \
      return hipErrorInvalidValue;         \
  }

// The fused kernel's launch for one number of x-y columns per thread C (each
// value compiled in a translation unit of its own, sos_fused.hip).
template <int C>
hipError_t launch_fused_cpt(const Dev& d, const SegLaunch& L, int fp32, int threads, size_t lds,
                            const FusedArgs& a, hipStream_t st, bool* plain);

}  // namespace sos
