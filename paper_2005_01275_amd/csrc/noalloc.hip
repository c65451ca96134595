// Fine-level residual evaluation that allocates no device memory.  The
// state and the residual in internal (renumbered) order live in a fixed
// file-scope device array instead of buffers allocated per call; every
// other buffer it touches belongs to the hierarchy, which was allocated
// when the hierarchy was built.
#include <mutex>

#include "hier.hpp"

namespace spfas {

// Two vectors of (flux + cell) unknowns: up to 6,291,456 unknowns of level 0
// (the 60x220x85 workload has 4,456,100).  Each device the library runs on
// holds this array until the process ends.
constexpr size_t kScratchDoubles = size_t(12) << 20;   // 96 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked
// up once per device.  In host code the array's name is not a device
// address: only this pointer may be handed to kernels or copies.
static double* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      fail(SPFAS_ERR_DEVICE, std::string("hipGetSymbolAddress of the residual scratch array failed: ") +
                                 hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

size_t noalloc_max_unknowns() { return kScratchDoubles / 2; }

void Hierarchy::eval_residual_noalloc(const double* p, const double* sig, double* rp, double* rs) {
  const int64_t n = fine.n, nf = fine.nf;
  if ((size_t)(nf + n) > noalloc_max_unknowns())
    fail(SPFAS_ERR_INVALID, "spfas_eval_residual_noalloc: " + std::to_string(nf + n) +
                                " level-0 unknowns exceed the scratch capacity of " +
                                std::to_string(noalloc_max_unknowns()));
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  require(dev >= 0 && dev < kMaxDevices, "device ordinal out of range");
  require(dev == device, "the current device is not the device the hierarchy was built on");
  double* x = scratch_on(dev);   // [nf + n] state, then [nf + n] residual
  double* r = x + (nf + n);
  hipStream_t s = stream;
  // every entry of x and r is written before it is read: nothing to clear
  launch_gather(nf, fine.flux_in.p, sig, x, s);
  launch_gather(n, fine.cell_in.p, p, x + nf, s);
  launch_fine_resid(fine.view(), x, nullptr, 0.0, r, parts.p, s);
  launch_fill(n_faces_in, 0.0, rs, s);
  launch_scatter(nf, fine.flux_in.p, r, rs, s);
  launch_scatter(n, fine.cell_in.p, r + nf, rp, s);
  HIPCHECK(hipStreamSynchronize(s));
}

}  // namespace spfas
