// Reduced-precision path on the gfx950 matrix cores.
//
// Complex products run as real MFMAs on an interleaved embedding: with the
// reduction index k carrying (re, im) pairs, a row of A is [Ar(k0) Ai(k0) ...]
// and the two real B operands are
//     Br' = [ Br(k)  ; -Bi(k) ]   -> real part of A*B
//     Bi' = [ Bi(k)  ;  Br(k) ]   -> imaginary part of A*B
// so one complex multiply-add costs four real ones (8 flops).
//
// Projection (Eq. proj_MB):  M[I][t] = sum_r U[I][r] F_t(r),
//   F_t(r) = conj(psi_occ[n][r]) psi_unocc[n'][r] formed while staging B tiles.
// Accumulation (Eq. polar_MB): P_j[I][J] += sum_t (w_j[t] M[I][t]) conj(M[J][t])
//   over lower tiles, FP32 accumulators for one chunk of pairs, then added into
//   the FP64 P (one owner per tile).
#include "gw_mfma.hpp"

#include <algorithm>

namespace gw {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128;          // tile rows (I)
constexpr int BN = 128;          // tile cols (pairs t, or J)
constexpr int KB = 16;           // complex k per LDS stage
constexpr int AS = 2 * KB + 1;   // floats per A row in LDS
constexpr int BS = 2 * KB + 2;   // floats per B column in LDS
constexpr int NT = 256;          // 4 waves: 2 x 2, each 64 x 64 complex
constexpr int LOADS = BM * KB / NT;  // staged elements per thread per operand (8)

__device__ inline void lower_tile(int l, int& bi, int& bj) {
  int b = (int)((sqrt(8.0 * (double)l + 1.0) - 1.0) * 0.5);
  while ((b + 1) * (b + 2) / 2 <= l) ++b;
  while (b * (b + 1) / 2 > l) --b;
  bi = b;
  bj = l - b * (b + 1) / 2;
}

struct AccF32 {
  floatx16 r[2][2];
  floatx16 i[2][2];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          r[a][b][v] = 0.f;
          i[a][b][v] = 0.f;
        }
  }
};

// One LDS stage of KB complex k: A rows [BM][AS], B columns [BN][BS].
__device__ inline void mma_stage_f32(const float* __restrict__ As, const float* __restrict__ Bs, AccF32& acc,
                                     int wm, int wn, int lane) {
  const int l32 = lane & 31, h = lane >> 5;
#pragma unroll 4
  for (int kk = 0; kk < KB; ++kk) {
    float a[2], br[2], bi[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) a[rb] = As[(wm * 64 + rb * 32 + l32) * AS + 2 * kk + h];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      float2 bv = *reinterpret_cast<const float2*>(&Bs[(wn * 64 + cb * 32 + l32) * BS + 2 * kk]);
      br[cb] = h ? -bv.y : bv.x;
      bi[cb] = h ? bv.x : bv.y;
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc.r[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rb], br[cb], acc.r[rb][cb], 0, 0, 0);
        acc.i[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rb], bi[cb], acc.i[rb][cb], 0, 0, 0);
      }
  }
}

// Element (row, col) of the wave tile held by (rb, cb, v) of this lane.
__device__ inline int acc_row(int wm, int rb, int v, int lane) {
  return wm * 64 + rb * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}
__device__ inline int acc_col(int wn, int cb, int lane) { return wn * 64 + cb * 32 + (lane & 31); }

// ---------------------------------------------------------------- projection
__global__ __launch_bounds__(NT, 2) void project_f32_kernel(int N, int R, const float2* __restrict__ U,
                                                            const float2* __restrict__ po,
                                                            const float2* __restrict__ pu, int no, int nu,
                                                            float2* __restrict__ M, long ldm) {
  __shared__ __attribute__((aligned(16))) float As[BM * AS];
  __shared__ __attribute__((aligned(16))) float Bs[BN * BS];
  const int T = no * nu;
  const int t0 = blockIdx.x * BN;
  const int i0 = blockIdx.y * BM;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int kq = tid % KB;        // k handled by this thread when staging
  const int rq = tid / KB;        // first staged row / pair (then +16 per load)

  // per-thread staging rows: A rows and (n, u) of B pairs
  const float2* arow[LOADS];
  const float2* orow[LOADS];
  const float2* urow[LOADS];
  bool aok[LOADS], bok[LOADS];
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    int gi = i0 + rq + 16 * q;
    aok[q] = gi < N;
    arow[q] = U + (size_t)(aok[q] ? gi : 0) * R;
    int gt = t0 + rq + 16 * q;
    bok[q] = gt < T;
    int t = bok[q] ? gt : 0;
    orow[q] = po + (size_t)(t / nu) * R;
    urow[q] = pu + (size_t)(t % nu) * R;
  }
  float2 ra[LOADS], ro[LOADS], ru[LOADS];
  auto gload = [&](int r0) {
    int r = r0 + kq;
    bool rok = r < R;
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      ra[q] = (aok[q] && rok) ? arow[q][r] : make_float2(0.f, 0.f);
      bool ok = bok[q] && rok;
      ro[q] = ok ? orow[q][r] : make_float2(0.f, 0.f);
      ru[q] = ok ? urow[q][r] : make_float2(0.f, 0.f);
    }
  };
  AccF32 acc;
  acc.zero();
  gload(0);
  for (int r0 = 0; r0 < R; r0 += KB) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      int row = rq + 16 * q;
      As[row * AS + 2 * kq] = ra[q].x;
      As[row * AS + 2 * kq + 1] = ra[q].y;
      // conj(o) * u
      float fr = ro[q].x * ru[q].x + ro[q].y * ru[q].y;
      float fi = ro[q].x * ru[q].y - ro[q].y * ru[q].x;
      *reinterpret_cast<float2*>(&Bs[row * BS + 2 * kq]) = make_float2(fr, fi);
    }
    __syncthreads();
    if (r0 + KB < R) gload(r0 + KB);
    mma_stage_f32(As, Bs, acc, wm, wn, lane);
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      int gt = t0 + acc_col(wn, cb, lane);
      if (gt >= T) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int gi = i0 + acc_row(wm, rb, v, lane);
        if (gi < N) M[(size_t)gi * ldm + gt] = make_float2(acc.r[rb][cb][v], acc.i[rb][cb][v]);
      }
    }
}

// ------------------------------------------------------------- accumulation
__global__ __launch_bounds__(NT, 2) void herk_f32_kernel(int N, int T, const float2* __restrict__ M, long ldm,
                                                         const float* __restrict__ w, double2* __restrict__ P) {
  __shared__ __attribute__((aligned(16))) float As[BM * AS];
  __shared__ __attribute__((aligned(16))) float Bs[BN * BS];
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int om = blockIdx.y;
  const float* wj = w + (size_t)om * T;
  const int i0 = bi * BM, j0 = bj * BN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int kq = tid % KB, rq = tid / KB;
  const float2* arow[LOADS];
  const float2* brow[LOADS];
  bool aok[LOADS], bok[LOADS];
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    int gi = i0 + rq + 16 * q, gj = j0 + rq + 16 * q;
    aok[q] = gi < N;
    bok[q] = gj < N;
    arow[q] = M + (size_t)(aok[q] ? gi : 0) * ldm;
    brow[q] = M + (size_t)(bok[q] ? gj : 0) * ldm;
  }
  float2 ra[LOADS], rb_[LOADS];
  float rw;
  auto gload = [&](int t0) {
    int t = t0 + kq;
    bool tok = t < T;
    rw = tok ? wj[t] : 0.f;
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      ra[q] = (aok[q] && tok) ? arow[q][t] : make_float2(0.f, 0.f);
      rb_[q] = (bok[q] && tok) ? brow[q][t] : make_float2(0.f, 0.f);
    }
  };
  AccF32 acc;
  acc.zero();
  gload(0);
  for (int t0 = 0; t0 < T; t0 += KB) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      int row = rq + 16 * q;
      As[row * AS + 2 * kq] = ra[q].x * rw;
      As[row * AS + 2 * kq + 1] = ra[q].y * rw;
      *reinterpret_cast<float2*>(&Bs[row * BS + 2 * kq]) = make_float2(rb_[q].x, -rb_[q].y);
    }
    __syncthreads();
    if (t0 + KB < T) gload(t0 + KB);
    mma_stage_f32(As, Bs, acc, wm, wn, lane);
  }
  double2* Pj = P + (size_t)om * N * N;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      int gj = j0 + acc_col(wn, cb, lane);
      if (gj >= N) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int gi = i0 + acc_row(wm, rb, v, lane);
        if (gi < N) {
          double2 p = Pj[(size_t)gi * N + gj];
          p.x += (double)acc.r[rb][cb][v];
          p.y += (double)acc.i[rb][cb][v];
          Pj[(size_t)gi * N + gj] = p;
        }
      }
    }
}

// w[j][t] = 4 D / (D^2 + w_j^2) evaluated in FP64, stored as float.
__global__ void weights_f32_kernel(const double* __restrict__ eps, int n_bands, int n_occ, Chunk c, OmegaList om,
                                   float* __restrict__ w) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int T = c.no * c.nu;
  if (t >= T) return;
  int n = c.n0 + t / c.nu;
  int u = c.u0 + t % c.nu;
  double d = eps[(size_t)c.k * n_bands + n] - eps[(size_t)c.kq * n_bands + n_occ + u];
  double d2 = d * d;
  for (int j = 0; j < om.n; ++j) w[(size_t)j * T + t] = (float)(4.0 * d / (d2 + om.w[j] * om.w[j]));
}

int launch_project_f32(hipStream_t s, int N, int R, const float2* U, const float2* po, const float2* pu, int no,
                       int nu, float2* M, long ldm) {
  int T = no * nu;
  dim3 grid((T + BN - 1) / BN, (N + BM - 1) / BM);
  ProfScope prof(s, "project_f32_kernel");
  hipLaunchKernelGGL(project_f32_kernel, grid, dim3(NT), 0, s, N, R, U, po, pu, no, nu, M, ldm);
  GW_LAUNCHED("project_f32_kernel");
  return GW_OK;
}


// ===================================================================== split 16-bit
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest even);
// a product is hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation.
// Complex numbers travel as one dword per word: (re, im) in the low/high half.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint32_t bits_of(bf16x2 v) { return __builtin_bit_cast(uint32_t, v); }

__device__ inline void split_bf16(float re, float im, uint32_t& hi, uint32_t& lo) {
  bf16x2 h = {(__bf16)re, (__bf16)im};
  float hr = (float)h[0], hm = (float)h[1];
  bf16x2 l = {(__bf16)(re - hr), (__bf16)(im - hm)};
  hi = bits_of(h);
  lo = bits_of(l);
}

constexpr int KS = 16;               // complex k per LDS stage (two MFMA k-steps of 8)
constexpr int SW = KS + 4;           // dwords per LDS row (padded)

struct Frag {
  uint4 v;
};

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
// (re, im) -> (re, -im): flips the sign bit of the high half of every dword
__device__ inline uint4 frag_conj(uint4 v) {
  return make_uint4(v.x ^ 0x80000000u, v.y ^ 0x80000000u, v.z ^ 0x80000000u, v.w ^ 0x80000000u);
}
// (re, im) -> (im, re)
__device__ inline uint32_t swap16(uint32_t x) { return (x >> 16) | (x << 16); }
__device__ inline uint4 frag_swap(uint4 v) { return make_uint4(swap16(v.x), swap16(v.y), swap16(v.z), swap16(v.w)); }

struct Lds16 {
  uint32_t ahi[BM * SW];
  uint32_t alo[BM * SW];
  uint32_t bhi[BN * SW];
  uint32_t blo[BN * SW];
};

__device__ inline void mma_stage_bf16(const Lds16& L, AccF32& acc, int wm, int wn, int lane) {
  const int l32 = lane & 31, h = lane >> 5;
#pragma unroll
  for (int s = 0; s < KS / 8; ++s) {
    const int off = s * 8 + h * 4;   // dword offset of this lane's 4 complex k
    uint4 ah[2], al[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      int row = wm * 64 + rb * 32 + l32;
      ah[rb] = *reinterpret_cast<const uint4*>(&L.ahi[row * SW + off]);
      al[rb] = *reinterpret_cast<const uint4*>(&L.alo[row * SW + off]);
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      int col = wn * 64 + cb * 32 + l32;
      uint4 bh = *reinterpret_cast<const uint4*>(&L.bhi[col * SW + off]);
      uint4 bl = *reinterpret_cast<const uint4*>(&L.blo[col * SW + off]);
      brh[cb] = frag_conj(bh);
      brl[cb] = frag_conj(bl);
      bih[cb] = frag_swap(bh);
      bil[cb] = frag_swap(bl);
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc.r[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ah[rb]), as_bf16x8(brh[cb]), acc.r[rb][cb], 0, 0, 0);
        acc.i[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ah[rb]), as_bf16x8(bih[cb]), acc.i[rb][cb], 0, 0, 0);
      }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc.r[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ah[rb]), as_bf16x8(brl[cb]), acc.r[rb][cb], 0, 0, 0);
        acc.i[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ah[rb]), as_bf16x8(bil[cb]), acc.i[rb][cb], 0, 0, 0);
      }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc.r[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(al[rb]), as_bf16x8(brh[cb]), acc.r[rb][cb], 0, 0, 0);
        acc.i[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(al[rb]), as_bf16x8(bih[cb]), acc.i[rb][cb], 0, 0, 0);
      }
  }
}

// U (c64 [N][R]) -> hi/lo words [N][Rp], zero beyond R (Rp = R rounded up to KS).
__global__ void split_u_bf16_kernel(int N, int R, int Rp, const float2* __restrict__ U, uint32_t* __restrict__ hi,
                                    uint32_t* __restrict__ lo) {
  size_t n = (size_t)N * Rp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e / Rp), r = (int)(e % Rp);
    float2 x = r < R ? U[(size_t)i * R + r] : make_float2(0.f, 0.f);
    uint32_t h, l;
    split_bf16(x.x, x.y, h, l);
    hi[e] = h;
    lo[e] = l;
  }
}

// Projection with pre-split U and products split while staging.
__global__ __launch_bounds__(NT, 1) void project_bf16_kernel(int N, int R, int Rp, const uint32_t* __restrict__ Uh,
                                                             const uint32_t* __restrict__ Ul,
                                                             const float2* __restrict__ po,
                                                             const float2* __restrict__ pu, int no, int nu,
                                                             float2* __restrict__ M, long ldm) {
  __shared__ __attribute__((aligned(16))) Lds16 L;
  const int T = no * nu;
  const int t0 = blockIdx.x * BN;
  const int i0 = blockIdx.y * BM;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  // A staging: 128 rows x 4 groups of 4 complex; two (row, group) slots per thread
  int arow_l[2], agrp[2];
  const uint32_t* ah_src[2];
  const uint32_t* al_src[2];
  bool aok[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int e = tid + q * NT;
    arow_l[q] = e >> 2;
    agrp[q] = e & 3;
    int gi = i0 + arow_l[q];
    aok[q] = gi < N;
    size_t base = (size_t)(aok[q] ? gi : 0) * Rp + agrp[q] * 4;
    ah_src[q] = Uh + base;
    al_src[q] = Ul + base;
  }
  // B staging as in the FP32 kernel: pair rq + 16 q, complex k kq
  const int kq = tid % KS, rq = tid / KS;
  const float2* orow[LOADS];
  const float2* urow[LOADS];
  bool bok[LOADS];
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    int gt = t0 + rq + 16 * q;
    bok[q] = gt < T;
    int t = bok[q] ? gt : 0;
    orow[q] = po + (size_t)(t / nu) * R;
    urow[q] = pu + (size_t)(t % nu) * R;
  }
  uint4 rah[2], ral[2];
  float2 ro[LOADS], ru[LOADS];
  auto gload = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      rah[q] = aok[q] ? *reinterpret_cast<const uint4*>(ah_src[q] + r0) : make_uint4(0, 0, 0, 0);
      ral[q] = aok[q] ? *reinterpret_cast<const uint4*>(al_src[q] + r0) : make_uint4(0, 0, 0, 0);
    }
    int r = r0 + kq;
    bool rok = r < R;
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      bool ok = bok[q] && rok;
      ro[q] = ok ? orow[q][r] : make_float2(0.f, 0.f);
      ru[q] = ok ? urow[q][r] : make_float2(0.f, 0.f);
    }
  };
  AccF32 acc;
  acc.zero();
  gload(0);
  for (int r0 = 0; r0 < R; r0 += KS) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<uint4*>(&L.ahi[arow_l[q] * SW + agrp[q] * 4]) = rah[q];
      *reinterpret_cast<uint4*>(&L.alo[arow_l[q] * SW + agrp[q] * 4]) = ral[q];
    }
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      int row = rq + 16 * q;
      float fr = ro[q].x * ru[q].x + ro[q].y * ru[q].y;
      float fi = ro[q].x * ru[q].y - ro[q].y * ru[q].x;
      uint32_t hh, ll;
      split_bf16(fr, fi, hh, ll);
      L.bhi[row * SW + kq] = hh;
      L.blo[row * SW + kq] = ll;
    }
    __syncthreads();
    if (r0 + KS < R) gload(r0 + KS);
    mma_stage_bf16(L, acc, wm, wn, lane);
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      int gt = t0 + acc_col(wn, cb, lane);
      if (gt >= T) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int gi = i0 + acc_row(wm, rb, v, lane);
        if (gi < N) M[(size_t)gi * ldm + gt] = make_float2(acc.r[rb][cb][v], acc.i[rb][cb][v]);
      }
    }
}

// Accumulation with both operands split while staging.
__global__ __launch_bounds__(NT, 2) void herk_bf16_kernel(int N, int T, const float2* __restrict__ M, long ldm,
                                                          const float* __restrict__ w, double2* __restrict__ P) {
  __shared__ __attribute__((aligned(16))) Lds16 L;
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int om = blockIdx.y;
  const float* wj = w + (size_t)om * T;
  const int i0 = bi * BM, j0 = bj * BN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int kq = tid % KS, rq = tid / KS;
  const float2* arow[LOADS];
  const float2* brow[LOADS];
  bool aok[LOADS], bok[LOADS];
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    int gi = i0 + rq + 16 * q, gj = j0 + rq + 16 * q;
    aok[q] = gi < N;
    bok[q] = gj < N;
    arow[q] = M + (size_t)(aok[q] ? gi : 0) * ldm;
    brow[q] = M + (size_t)(bok[q] ? gj : 0) * ldm;
  }
  float2 ra[LOADS], rb_[LOADS];
  float rw;
  auto gload = [&](int t0) {
    int t = t0 + kq;
    bool tok = t < T;
    rw = tok ? wj[t] : 0.f;
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      ra[q] = (aok[q] && tok) ? arow[q][t] : make_float2(0.f, 0.f);
      rb_[q] = (bok[q] && tok) ? brow[q][t] : make_float2(0.f, 0.f);
    }
  };
  AccF32 acc;
  acc.zero();
  gload(0);
  for (int t0 = 0; t0 < T; t0 += KS) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      int row = rq + 16 * q;
      uint32_t hh, ll;
      split_bf16(ra[q].x * rw, ra[q].y * rw, hh, ll);
      L.ahi[row * SW + kq] = hh;
      L.alo[row * SW + kq] = ll;
      split_bf16(rb_[q].x, -rb_[q].y, hh, ll);
      L.bhi[row * SW + kq] = hh;
      L.blo[row * SW + kq] = ll;
    }
    __syncthreads();
    if (t0 + KS < T) gload(t0 + KS);
    mma_stage_bf16(L, acc, wm, wn, lane);
  }
  double2* Pj = P + (size_t)om * N * N;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      int gj = j0 + acc_col(wn, cb, lane);
      if (gj >= N) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int gi = i0 + acc_row(wm, rb, v, lane);
        if (gi < N) {
          double2 p = Pj[(size_t)gi * N + gj];
          p.x += (double)acc.r[rb][cb][v];
          p.y += (double)acc.i[rb][cb][v];
          Pj[(size_t)gi * N + gj] = p;
        }
      }
    }
}

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

int launch_split_u_bf16(hipStream_t s, int N, int R, int Rp, const float2* U, uint32_t* hi, uint32_t* lo) {
  size_t n = (size_t)N * Rp;
  unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(split_u_bf16_kernel, dim3(blocks), dim3(256), 0, s, N, R, Rp, U, hi, lo);
  GW_LAUNCHED("split_u_bf16_kernel");
  return GW_OK;
}

int launch_project_bf16(hipStream_t s, int N, int R, int Rp, const uint32_t* Uh, const uint32_t* Ul, const float2* po,
                        const float2* pu, int no, int nu, float2* M, long ldm) {
  int T = no * nu;
  dim3 grid((T + BN - 1) / BN, (N + BM - 1) / BM);
  ProfScope prof(s, "project_bf16_kernel");
  hipLaunchKernelGGL(project_bf16_kernel, grid, dim3(NT), 0, s, N, R, Rp, Uh, Ul, po, pu, no, nu, M, ldm);
  GW_LAUNCHED("project_bf16_kernel");
  return GW_OK;
}

}  // namespace

int mfma_default_chunk_pairs(int N, int precision) {
  (void)precision;
  size_t target = (size_t)192 << 20;  // M chunk bytes (c64)
  size_t p = target / ((size_t)N * 8);
  p = std::max<size_t>(BN, std::min<size_t>(p, 4096));
  return (int)p;
}

void mfma_adjust_chunk(int, int&, int&, int, int) {}

static size_t split_u_bytes(int precision, int N, int R) {
  if (precision == GW_FP32) return 0;
  size_t Rp = (size_t)round_up(R, KS);
  return 2 * align_up((size_t)N * Rp * sizeof(uint32_t));
}

size_t mfma_pol_workspace(int precision, int N, int R, int tc, int n_omega) {
  return split_u_bytes(precision, N, R) + align_up((size_t)N * tc * sizeof(float2)) +
         align_up((size_t)n_omega * tc * sizeof(float));
}

size_t mfma_project_workspace(int precision, int N, int R, int n_occ, int n_unocc) {
  (void)n_occ;
  (void)n_unocc;
  return split_u_bytes(precision, N, R);
}

int mfma_project(hipStream_t s, int precision, int N, int R, int n_occ, int n_unocc, const void* U,
                 const void* psi_occ, const void* psi_unocc, void* M, void* ws, size_t ws_bytes) {
  (void)ws_bytes;
  if (precision == GW_FP32)
    return launch_project_f32(s, N, R, static_cast<const float2*>(U), static_cast<const float2*>(psi_occ),
                              static_cast<const float2*>(psi_unocc), n_occ, n_unocc, static_cast<float2*>(M),
                              (long)n_occ * n_unocc);
  if (precision != GW_SPLIT_BF16) return fail(GW_ERR_UNSUPPORTED, "gw_project: precision not built yet");
  const int Rp = round_up(R, KS);
  Carver cv(ws);
  uint32_t* Uh = cv.take<uint32_t>((size_t)N * Rp);
  uint32_t* Ul = cv.take<uint32_t>((size_t)N * Rp);
  int st = launch_split_u_bf16(s, N, R, Rp, static_cast<const float2*>(U), Uh, Ul);
  if (st != GW_OK) return st;
  return launch_project_bf16(s, N, R, Rp, Uh, Ul, static_cast<const float2*>(psi_occ),
                             static_cast<const float2*>(psi_unocc), n_occ, n_unocc, static_cast<float2*>(M),
                             (long)n_occ * n_unocc);
}

int mfma_polarization(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                      const OmegaList& om, void* ws) {
  if (d.precision != GW_FP32 && d.precision != GW_SPLIT_BF16)
    return fail(GW_ERR_UNSUPPORTED, "gw_polarization: precision not built yet");
  Carver cv(ws);
  const int Rp = round_up(d.R, KS);
  uint32_t* Uh = nullptr;
  uint32_t* Ul = nullptr;
  if (d.precision == GW_SPLIT_BF16) {
    Uh = cv.take<uint32_t>((size_t)d.N * Rp);
    Ul = cv.take<uint32_t>((size_t)d.N * Rp);
  }
  float2* M = cv.take<float2>((size_t)d.N * tc);
  float* w = cv.take<float>((size_t)d.n_omega * tc);
  const float2* U = static_cast<const float2*>(d.U);
  const float2* psi = static_cast<const float2*>(d.psi);
  const int nb = d.n_occ + d.n_unocc;
  const int ntile = (d.N + BM - 1) / BM;
  double2* P = reinterpret_cast<double2*>(d.P);
  if (d.precision == GW_SPLIT_BF16) {
    int st = launch_split_u_bf16(s, d.N, d.R, Rp, U, Uh, Ul);
    if (st != GW_OK) return st;
  }
  for (const Chunk& c : chunks) {
    const int T = c.pairs();
    hipLaunchKernelGGL(weights_f32_kernel, dim3((T + 255) / 256), dim3(256), 0, s, d.eps, nb, d.n_occ, c, om, w);
    GW_LAUNCHED("weights_f32_kernel");
    const float2* po = psi + ((size_t)c.k * nb + c.n0) * d.R;
    const float2* pu = psi + ((size_t)c.kq * nb + d.n_occ + c.u0) * d.R;
    dim3 hgrid(ntile * (ntile + 1) / 2, d.n_omega);
    if (d.precision == GW_FP32) {
      int st = launch_project_f32(s, d.N, d.R, U, po, pu, c.no, c.nu, M, T);
      if (st != GW_OK) return st;
      ProfScope prof(s, "herk_f32_kernel");
      hipLaunchKernelGGL(herk_f32_kernel, hgrid, dim3(NT), 0, s, d.N, T, M, (long)T, w, P);
      GW_LAUNCHED("herk_f32_kernel");
    } else {
      int st = launch_project_bf16(s, d.N, d.R, Rp, Uh, Ul, po, pu, c.no, c.nu, M, T);
      if (st != GW_OK) return st;
      ProfScope prof(s, "herk_bf16_kernel");
      hipLaunchKernelGGL(herk_bf16_kernel, hgrid, dim3(NT), 0, s, d.N, T, M, (long)T, w, P);
      GW_LAUNCHED("herk_bf16_kernel");
    }
  }
  return GW_OK;
}

}  // namespace gw
