// kx1.hip -- gradient-mode instantiations of the screened quartet engine;
// see kx_impl.h.
#include "kx_impl.h"

namespace mderi {

hipError_t launch_kx_grad(const KxArgs &a, int npt, int Lmax, int waves, size_t lds, int grid, hipStream_t s) {
  return kx::launch_mode<1>(a, npt, Lmax, waves, lds, grid, s);
}

}  // namespace mderi
