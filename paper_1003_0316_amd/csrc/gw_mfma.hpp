// Reduced-precision (FP32 / split-BF16 / split-FP16) matrix-core path.
#pragma once

#include <vector>

#include "gw_internal.hpp"

namespace gw {

int mfma_default_chunk_pairs(int N, int precision);
size_t mfma_pol_workspace(int precision, int N, int R, int tc, int n_omega);
size_t mfma_project_workspace(int precision, int N, int R, int n_occ, int n_unocc);
int mfma_project(hipStream_t s, int precision, int N, int R, int n_occ, int n_unocc, const void* U,
                 const void* psi_occ, const void* psi_unocc, void* M, void* ws, size_t ws_bytes);
int mfma_polarization(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                      const OmegaList& om, void* ws);

}  // namespace gw
