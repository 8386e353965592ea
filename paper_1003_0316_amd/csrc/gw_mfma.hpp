// Reduced-precision (FP32 / split-BF16 / split-FP16) matrix-core path.
#pragma once

#include <vector>

#include "gw_internal.hpp"

namespace gw {

int mfma_default_chunk_pairs(int N, int R, int n_omega, int precision);
size_t mfma_pol_workspace(int precision, int N, int R, int tc, int n_omega, size_t psi_rows);
size_t mfma_project_workspace(int precision, int N, int R, int n_occ, int n_unocc);
int mfma_project(hipStream_t s, int precision, int N, int R, int n_occ, int n_unocc, const void* U,
                 const void* psi_occ, const void* psi_unocc, void* M, void* ws, size_t ws_bytes);
int mfma_polarization(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                      const OmegaList& om, void* ws);

// Split-BF16 on pre-tiled operands (k_tiled.hip).
extern int g_bf16_pipeline;   // 1: operands staged inside the GEMM kernels; 2: pre-tiled operands
extern int g_gemm_staging;    // pre-tiled GEMM core: 1 through registers, 2 direct global -> LDS
extern int g_complex_product; // pre-tiled pipeline: 4 real products per complex product, or 3 (Gauss form)
extern int g_real_core;       // real inputs: 1 the 8-wave register-staged core, 2 the six-slot core
extern int g_gemm3m_lead;     // six-slot ring: plane steps between a slot's copy and its use (3..5)
extern int g_gemm3m_pipeline; // three-product core staging: 2 stage buffers, or 6 plane slots
extern int g_fp16_core;       // split FP16: 1 operands staged inside the GEMM kernels, 2 the three-product core
size_t tiled_pol_workspace(int N, int R, int tc, int n_omega, size_t psi_rows);
size_t tiled_project_workspace(int N, int R, int n_occ, int n_unocc);
// Split FP16 on the three-multiplication core (power-of-two scaled plane words).
int tiled_polarization_f16(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                           const OmegaList& om, void* ws);
int tiled_project_f16(hipStream_t s, int N, int R, int n_occ, int n_unocc, const float2* U, const float2* po,
                      const float2* pu, float2* M, void* ws);
int tiled_default_chunk_pairs(int N, int R, int n_omega);
int tiled_project(hipStream_t s, int N, int R, int n_occ, int n_unocc, const float2* U, const float2* po,
                  const float2* pu, float2* M, void* ws);
int tiled_polarization(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                       const OmegaList& om, void* ws);

// Real inputs (inversion-symmetric case), split BF16 (k_tiled.hip).
size_t tiled_pol_workspace_real(int N, int R, int tc, int n_omega);
int tiled_polarization_real(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                            const OmegaList& om, void* ws);

// Correlation self-energy, split-BF16 quadratic forms (k_tiled.hip) for a
// batch of g states sharing one momentum transfer: q [n_mesh][cols], the
// states' columns side by side, cols = tiled_sigma_cols(nb, g), state i at
// column i * cols / g.
int tiled_sigma_cols(int nb, int g);
size_t tiled_sigma_workspace(int N, int R, int nb, int g);
int tiled_sigma_quadforms(hipStream_t s, int N, int R, int nb, int g, int n_mesh, const float2* U, bool tile_u,
                          const float2* const* psi_state, const float2* const* psi_all, const double2* W,
                          const double* v, double* q, void* ws);

}  // namespace gw
