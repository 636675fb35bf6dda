// kx0.hip -- digest-mode instantiations of the screened quartet engine
// (K and J builds) and its launcher; see kx_impl.h.
#include "kx_impl.h"

namespace mderi {

hipError_t launch_kx_grad(const KxArgs &a, int npt, int Lmax, int waves, size_t lds, int grid, hipStream_t s);

hipError_t launch_kx(const KxArgs &a, int npt, int Lmax, bool grad, int waves, size_t lds, int grid, hipStream_t s) {
  if (a.nchunk <= 0) return hipSuccess;
  if (waves < 1 || waves > kx::kWavesMax || grid <= 0 || lds > 160 * 1024) return hipErrorInvalidValue;
  if (grad) return launch_kx_grad(a, npt, Lmax, waves, lds, grid, s);
  return kx::launch_mode<0>(a, npt, Lmax, waves, lds, grid, s);
}

}  // namespace mderi
