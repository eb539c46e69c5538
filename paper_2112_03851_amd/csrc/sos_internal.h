// Internal descriptors shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sos {

constexpr int kMaxPlane = 4096;   // max x-y node plane of a subdomain
constexpr int kMaxCols = 8;       // max x-y columns per thread in a z-march
constexpr int kPad = 2;           // zero padding around an LDS plane (stencil radius)

// One subdomain: a box of elements. Its unknowns are the kept nodes of the
// closed box (outer Dirichlet planes removed), numbered along its local axes
// 0 (fastest), 1, 2 (the marched axis): local axis a is global axis perm[a].
// Fields marked "local" are in local axis order, the others in global order.
struct SubDesc {
  int64_t off;      // offset of local node 0 in the concatenated vectors
  int32_t n[3];     // local: kept nodes per axis
  int32_t klo[3];   // local: closure index (0..2*ne) of local node 0 per axis
  int32_t ne2[3];   // local: 2 * elements per axis = closure index of the last node
  int32_t lo[3];    // global: global node index of local node 0 per axis
  int32_t pidx[3];  // global: position in the partition grid
  int32_t e0[3];    // global: first element per axis
  int32_t face[6];  // local: directed face (s <- j) id for (axis, side), -1 if none
  int32_t perm[3];  // global axis of local axis a
  int32_t iperm[3]; // local axis of global axis g
  int32_t tswap;    // bit a: the Robin datum of a local-axis-a face runs along its
                    // second local tangential axis fastest (global axis order)
  int32_t pad;
  double ks[3];     // local: 1/(3h) per axis (scale of the 1D stiffness stencil)
  double ms[3];     // local: h/30 per axis (scale of the 1D mass stencil)
  double elo[3];    // local: Robin coefficient at closure node 0 per axis (0 if none)
  double ehi[3];    // local: Robin coefficient at closure node ne2 per axis
  double qlo[3];    // local: second-order coefficient q at closure node 0 per axis (0 if none)
  double qhi[3];    // local: second-order coefficient q at closure node ne2 per axis
  int32_t copy;     // index of the problem copy this subdomain belongs to (batched copies)
  int32_t sbase;    // index of that copy's first subdomain
  int64_t xoff;     // offset of its x-boundary right-hand side: 2 n1 n2 values, the
                    // nodes i = 0, then i = n0 - 1, node (j, k) at j + n1 k
};

// One directed face (s <- j).
struct FaceDesc {
  int64_t lam_off;  // offset of its datum in the lambda array
  int32_t s, j, axis, side;
  int32_t na, nb;   // tangential extents (first tangential axis fastest)
  int32_t opp;      // id of (j <- s)
  double p;         // Robin coefficient p_sj
  double q;         // second-order coefficient q_sj (0: zeroth order)
};

// Geometry shared by all kernels.
struct Geom {
  double h[3];       // element sizes
  double ks[3];      // 1/(3h): scale of the integer 1D stiffness stencil
  double ms[3];      // h/30:   scale of the integer 1D mass stencil
  int32_t ne[3];
  int32_t nn[3];     // global nodes per axis (2ne+1)
  int32_t nparts[3];
  int32_t n_sub;      // subdomains of all copies
  int32_t copies;     // independent copies of the problem (1 unless batched)
  int32_t bc[6];
};

// Per-subdomain scalars of the inner CG (FP64).
struct CgScal {
  double rz[2];      // r'z of the last two iterations (ping-pong by parity)
  double rr0;        // ||r_0||^2 of the current inner solve
  double stop2;      // squared stopping threshold
  int32_t done;      // inner solve finished
  int32_t iters;     // CG iterations of the current inner solve
  int32_t breakdown; // p'Ap <= 0 or non-finite
  int32_t pad;
};

}  // namespace sos
