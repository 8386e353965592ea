#include "gw_mfma.hpp"

namespace gw {

int mfma_default_chunk_pairs(int, int) { return 4096; }
void mfma_adjust_chunk(int, int&, int&, int, int) {}
size_t mfma_pol_workspace(int, int, int, int, int) { return 0; }
size_t mfma_project_workspace(int, int, int, int, int) { return 0; }
int mfma_project(hipStream_t, int, int, int, int, int, const void*, const void*, const void*, void*, void*,
                 size_t) {
  return fail(GW_ERR_UNSUPPORTED, "reduced-precision projection not built yet");
}
int mfma_polarization(hipStream_t, const gw_pol_desc&, const std::vector<Chunk>&, int, const OmegaList&, void*) {
  return fail(GW_ERR_UNSUPPORTED, "reduced-precision polarization not built yet");
}

}  // namespace gw
