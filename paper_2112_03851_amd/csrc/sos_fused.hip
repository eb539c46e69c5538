// Launches of the fused CG kernel for one number of x-y columns per thread,
// SOS_FUSED_CPT (this file is compiled once per value: the kernel variants
// of one value are independent of the others').
#include "sos_device.h"

#ifndef SOS_FUSED_CPT
#error SOS_FUSED_CPT must be defined (1..4)
#endif

namespace sos {

// True when the device's compute units can hold all `blocks` blocks of the
// kernel at once (occupancy of the kernel alone, dynamic LDS included). The
// answer for the last (device, kernel, shape) is kept per host thread: the
// same launch repeats every outer iteration.
static bool team_grid_resident(const void* fn, int threads, size_t lds, int blocks) {
  struct Memo {
    int dev = -1, threads = 0, blocks = 0;
    const void* fn = nullptr;
    size_t lds = 0;
    bool ok = false;
  };
  static thread_local Memo memo;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (memo.dev == dev && memo.fn == fn && memo.threads == threads && memo.lds == lds && memo.blocks == blocks)
    return memo.ok;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return false;
  memo = {dev, threads, blocks, fn, lds, (long long)per_cu * cus >= blocks};
  return memo.ok;
}

template <typename T, int C, bool Q, bool ZU, int RES = 0>
static hipError_t fused_launch_one(const Dev& d, const SegLaunch& L, int threads, size_t lds, const FusedArgs& a,
                                   hipStream_t st, bool* plain) {
  const dim3 grid(a.nblocks), block(threads);
  if (plain) {  // query only: would the launch be a plain one?
    *plain = a.team <= 1 ||
             team_grid_resident((const void*)k_fused_cg<T, C, Q, ZU, true, RES>, threads, lds, (int)grid.x);
    return hipSuccess;
  }
  if (a.team <= 1) {
    hipLaunchKernelGGL((k_fused_cg<T, C, Q, ZU, false, RES>), grid, block, lds, st, d, L.bfirst, a);
    return hipGetLastError();
  }
  // team barriers spin: every block of the grid must be resident at once.
  // When the occupancy of the kernel alone admits the whole grid, a plain
  // launch dispatches every block at once (and can be captured in a graph);
  // otherwise the cooperative launch checks residency and fails instead. A
  // member that still waits too long reports a failed barrier.
  const void* fn = (const void*)k_fused_cg<T, C, Q, ZU, true, RES>;
  if (team_grid_resident(fn, threads, lds, (int)grid.x)) {
    hipLaunchKernelGGL((k_fused_cg<T, C, Q, ZU, true, RES>), grid, block, lds, st, d, L.bfirst, a);
    return hipGetLastError();
  }
  Dev dd = d;
  const int32_t* bf = L.bfirst;
  FusedArgs aa = a;
  void* args[] = {&dd, &bf, &aa};
  const hipError_t e = hipLaunchCooperativeKernel(fn, grid, block, args, (unsigned)lds, st);
  // the error is returned here: clear HIP's per-thread last error too, or the
  // next launch check of any problem on this thread would report it again
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

template <int C>
hipError_t launch_fused_cpt(const Dev& d, const SegLaunch& L, int fp32, int threads, size_t lds,
                            const FusedArgs& a, hipStream_t st, bool* plain) {
  SOS_DISPATCH_Q(d.hasq, {
    if (fp32 && a.zu && a.res == 1) {
      return (fused_launch_one<float, C, Q, true, 1>(d, L, threads, a.lds_bytes, a, st, plain));
    } else if (fp32 && a.zu && a.res == 2) {
      return (fused_launch_one<float, C, Q, true, 2>(d, L, threads, a.lds_bytes, a, st, plain));
    } else if (fp32 && a.zu) {
      return (fused_launch_one<float, C, Q, true>(d, L, threads, lds, a, st, plain));
    } else if (fp32) {
      return (fused_launch_one<float, C, Q, false>(d, L, threads, lds, a, st, plain));
    } else if (a.zu) {
      return (fused_launch_one<double, C, Q, true>(d, L, threads, lds, a, st, plain));
    } else {
      return (fused_launch_one<double, C, Q, false>(d, L, threads, lds, a, st, plain));
    }
  });
  return hipSuccess;
}

template hipError_t launch_fused_cpt<SOS_FUSED_CPT>(const Dev&, const SegLaunch&, int, int, size_t,
                                                    const FusedArgs&, hipStream_t, bool*);

}  // namespace sos
