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
#include <string>

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
                                                            const float2* __restrict__ pu, int nu, long tb, int T,
                                                            float2* __restrict__ M, long ldm) {
  __shared__ __attribute__((aligned(16))) float As[BM * AS];
  __shared__ __attribute__((aligned(16))) float Bs[BN * BS];
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
    const long g = tb + t;
    orow[q] = po + (size_t)(g / nu) * R;
    urow[q] = pu + (size_t)(g % nu) * R;
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

// w[j][t] = pair_weight (as in the FP64 path) evaluated in FP64, stored as float.
__global__ void weights_f32_kernel(const double* __restrict__ eps, int n_bands, int n_occ, Chunk c, OmegaList om,
                                   float* __restrict__ w) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int T = c.T;
  if (t >= T) return;
  long g = c.tb + t;
  int n = c.n0 + (int)(g / c.nu);
  int u = c.u0 + (int)(g % c.nu);
  double d = eps[(size_t)c.k * n_bands + n] - eps[(size_t)c.kq * n_bands + n_occ + u];
  for (int j = 0; j < om.n; ++j) w[(size_t)j * T + t] = (float)pair_weight(d, om, j);
}

int launch_project_f32(hipStream_t s, int N, int R, const float2* U, const float2* po, const float2* pu, int nu,
                       long tb, int T, float2* M, long ldm) {
  dim3 grid((T + BN - 1) / BN, (N + BM - 1) / BM);
  ProfScope prof(s, "project_f32_kernel");
  hipLaunchKernelGGL(project_f32_kernel, grid, dim3(NT), 0, s, N, R, U, po, pu, nu, tb, T, M, ldm);
  GW_LAUNCHED("project_f32_kernel");
  return GW_OK;
}


// ===================================================================== split 16-bit
// Every FP32 operand x is carried as two 16-bit words.
//   BF16: hi = bf16(x), lo = bf16(x - hi); a product is hi*hi + hi*lo + lo*hi
//         accumulated in one FP32 accumulator.
//   FP16: x is first scaled by a power of two s (so that max|x s| lies in
//         [2^13, 2^14), inside FP16's normal range); hi = f16(x s) and
//         lo = f16((x s - hi) 2^11); hi*hi goes to one accumulator and
//         hi*lo + lo*hi to a second, combined as (acc + 2^-11 acc2) / (s_a s_b).
// Rounding is to nearest even in both formats.  Complex numbers travel as one
// dword per word: (re, im) in the low/high half.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// Operand words: BF16 hi + lo; FP16 hi + lo (power-of-two scaled, lo kept in
// range by 2^11 and accumulated apart); FP16 hi alone (the single-precision
// ablation: same scaling, no lo words and no correction products).
enum Word { W_BF16 = 0, W_F16 = 1, W_F16S = 2 };
constexpr bool is_f16(int w) { return w != W_BF16; }

template <int WORD>
__device__ inline void split_word(float re, float im, float s, uint32_t& hi, uint32_t& lo) {
  if constexpr (WORD == W_BF16) {
    bf16x2 h = {(__bf16)re, (__bf16)im};
    bf16x2 l = {(__bf16)(re - (float)h[0]), (__bf16)(im - (float)h[1])};
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, l);
  } else {
    float a = re * s, b = im * s;
    halfx2 h = {(_Float16)a, (_Float16)b};
    hi = __builtin_bit_cast(uint32_t, h);
    if constexpr (WORD == W_F16) {
      halfx2 l = {(_Float16)((a - (float)h[0]) * 2048.f), (_Float16)((b - (float)h[1]) * 2048.f)};
      lo = __builtin_bit_cast(uint32_t, l);
    } else {
      lo = 0u;
    }
  }
}

template <int WORD>
__device__ inline floatx16 mma16(uint4 a, uint4 b, floatx16 c) {
  if constexpr (!is_f16(WORD))
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c, 0,
                                                  0, 0);
}

// power of two s with max*s in [2^13, 2^14) (1 if max is 0 or not finite)
__device__ inline float pow2_scale(float mx) {
  if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
  int e;
  frexpf(mx, &e);  // mx = m 2^e, m in [0.5, 1)
  return ldexpf(1.f, 14 - e);
}

constexpr int KS = 16;               // complex k per LDS stage (two MFMA k-steps of 8)
constexpr int SW = KS + 4;           // dwords per LDS row (padded)

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

// Device-side scale bookkeeping of the FP16 words (maxima as float bit
// patterns; non-negative floats order like their bit patterns).
struct Scales {
  unsigned u, psi, m;
  unsigned w[kMaxOmega];
};

__device__ inline void atomic_max_pos(unsigned* p, float v) { atomicMax(p, __float_as_uint(v)); }

template <int WORD>
__device__ inline void mma_stage16(const Lds16& L, AccF32& acc, AccF32& acc2, int wm, int wn, int lane) {
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
        acc.r[rb][cb] = mma16<WORD>(ah[rb], brh[cb], acc.r[rb][cb]);
        acc.i[rb][cb] = mma16<WORD>(ah[rb], bih[cb], acc.i[rb][cb]);
      }
    if constexpr (WORD == W_F16S) continue;
    AccF32& c2 = (WORD == W_BF16) ? acc : acc2;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        c2.r[rb][cb] = mma16<WORD>(ah[rb], brl[cb], c2.r[rb][cb]);
        c2.i[rb][cb] = mma16<WORD>(ah[rb], bil[cb], c2.i[rb][cb]);
      }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        c2.r[rb][cb] = mma16<WORD>(al[rb], brh[cb], c2.r[rb][cb]);
        c2.i[rb][cb] = mma16<WORD>(al[rb], bih[cb], c2.i[rb][cb]);
      }
  }
}

// max |component| of a c64 array (FP16 scale of U and psi).
__global__ void maxabs_kernel(const float2* __restrict__ x, size_t n, unsigned* __restrict__ out) {
  __shared__ float red[256];
  float m = 0.f;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    float2 v = x[e];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomic_max_pos(out, red[0]);
}

__global__ void zero_u32_kernel(unsigned* __restrict__ p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// U (c64 [N][R]) -> hi/lo words [N][Rp], zero beyond R (Rp = R rounded up to KS).
template <int WORD>
__global__ void split_u_kernel(int N, int R, int Rp, const float2* __restrict__ U, const Scales* __restrict__ sc,
                               uint32_t* __restrict__ hi, uint32_t* __restrict__ lo) {
  const float s = is_f16(WORD) ? pow2_scale(__uint_as_float(sc->u)) : 1.f;
  size_t n = (size_t)N * Rp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e / Rp), r = (int)(e % Rp);
    float2 x = r < R ? U[(size_t)i * R + r] : make_float2(0.f, 0.f);
    uint32_t h, l;
    split_word<WORD>(x.x, x.y, s, h, l);
    hi[e] = h;
    lo[e] = l;
  }
}

// Projection with pre-split U and products split while staging.
template <int WORD>
__global__ __launch_bounds__(NT, WORD == W_F16 ? 1 : 2) void project16_kernel(int N, int R, int Rp, const uint32_t* __restrict__ Uh,
                                                          const uint32_t* __restrict__ Ul,
                                                          const float2* __restrict__ po,
                                                          const float2* __restrict__ pu, int nu, long tb, int T,
                                                          float2* __restrict__ M, long ldm, Scales* __restrict__ sc) {
  __shared__ __attribute__((aligned(16))) Lds16 L;
  const int t0 = blockIdx.x * BN;
  const int i0 = blockIdx.y * BM;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  float sF = 1.f, unscale = 1.f;
  if constexpr (is_f16(WORD)) {
    const float mp = __uint_as_float(sc->psi);
    sF = pow2_scale(2.f * mp * mp);
    unscale = 1.f / (pow2_scale(__uint_as_float(sc->u)) * sF);
  }
  // A staging: 128 rows x 4 groups of 4 complex; two (row, group) slots per
  // thread.  Offsets are 32-bit and relative to the tile's first row (rows past
  // N read the tile's first row and are zeroed), so the kernel fits two waves
  // per SIMD.
  const uint32_t* UhT = Uh + (size_t)i0 * Rp;
  const uint32_t* UlT = Ul + (size_t)i0 * Rp;
  int arow_l[2], agrp[2];
  uint32_t asrc[2], amask[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int e = tid + q * NT;
    arow_l[q] = e >> 2;
    agrp[q] = e & 3;
    int gi = i0 + arow_l[q];
    amask[q] = gi < N ? 0xffffffffu : 0u;
    asrc[q] = (uint32_t)((size_t)((gi < N ? gi : i0) - i0) * Rp + agrp[q] * 4);
  }
  // B staging as in the FP32 kernel: pair rq + 16 q, complex k kq
  const int kq = tid % KS, rq = tid / KS;
  uint32_t ooff[LOADS], uoff[LOADS];
  float bmask[LOADS];
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    int gt = t0 + rq + 16 * q;
    bmask[q] = gt < T ? 1.f : 0.f;
    int t = gt < T ? gt : 0;
    const long g = tb + t;
    ooff[q] = (uint32_t)((size_t)(g / nu) * R);
    uoff[q] = (uint32_t)((size_t)(g % nu) * R);
  }
  uint4 rah[2], ral[2];
  float2 ro[LOADS], ru[LOADS];
  float rmask = 1.f;
  auto gload = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      uint4 x = *reinterpret_cast<const uint4*>(UhT + asrc[q] + r0);
      uint4 y = *reinterpret_cast<const uint4*>(UlT + asrc[q] + r0);
      x.x &= amask[q]; x.y &= amask[q]; x.z &= amask[q]; x.w &= amask[q];
      y.x &= amask[q]; y.y &= amask[q]; y.z &= amask[q]; y.w &= amask[q];
      rah[q] = x;
      ral[q] = y;
    }
    int r = r0 + kq;
    rmask = r < R ? 1.f : 0.f;
    r = r < R ? r : R - 1;
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      float m = bmask[q] * rmask;
      float2 o = po[ooff[q] + r], u = pu[uoff[q] + r];
      ro[q] = make_float2(o.x * m, o.y * m);
      ru[q] = u;
    }
  };
  AccF32 acc, acc2;
  acc.zero();
  if constexpr (WORD == W_F16) acc2.zero();
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
      split_word<WORD>(fr, fi, sF, hh, ll);
      L.bhi[row * SW + kq] = hh;
      L.blo[row * SW + kq] = ll;
    }
    __syncthreads();
    if (r0 + KS < R) gload(r0 + KS);
    mma_stage16<WORD>(L, acc, acc2, wm, wn, lane);
  }
  float mloc = 0.f;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      int gt = t0 + acc_col(wn, cb, lane);
      if (gt >= T) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int gi = i0 + acc_row(wm, rb, v, lane);
        if (gi < N) {
          float re = acc.r[rb][cb][v], im = acc.i[rb][cb][v];
          if constexpr (WORD == W_F16) {
            re += acc2.r[rb][cb][v] * (1.f / 2048.f);
            im += acc2.i[rb][cb][v] * (1.f / 2048.f);
          }
          if constexpr (is_f16(WORD)) {
            re *= unscale;
            im *= unscale;
            mloc = fmaxf(mloc, fmaxf(fabsf(re), fabsf(im)));
          }
          M[(size_t)gi * ldm + gt] = make_float2(re, im);
        }
      }
    }
  if constexpr (is_f16(WORD)) {
    // block maximum of |M| for the accumulation's scale
    __shared__ float red[NT];
    red[tid] = mloc;
    __syncthreads();
    for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
      if (tid < s2) red[tid] = fmaxf(red[tid], red[tid + s2]);
      __syncthreads();
    }
    if (tid == 0 && sc) atomic_max_pos(&sc->m, red[0]);
  }
}

// Accumulation with both operands split while staging.
template <int WORD>
__global__ __launch_bounds__(NT, WORD == W_F16 ? 1 : 2) void herk16_kernel(int N, int T, const float2* __restrict__ M,
                                                                            long ldm, const float* __restrict__ w,
                                                                            double2* __restrict__ P,
                                                                            const Scales* __restrict__ sc) {
  __shared__ __attribute__((aligned(16))) Lds16 L;
  int bi, bj;
  lower_tile(blockIdx.x, bi, bj);
  const int om = blockIdx.y;
  const float* wj = w + (size_t)om * T;
  const int i0 = bi * BM, j0 = bj * BN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  float sA = 1.f, sB = 1.f, unscale = 1.f;
  if constexpr (is_f16(WORD)) {
    const float mm = __uint_as_float(sc->m);
    sA = pow2_scale(mm * __uint_as_float(sc->w[om]));
    sB = pow2_scale(mm);
    unscale = 1.f / (sA * sB);
  }
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
  AccF32 acc, acc2;
  acc.zero();
  if constexpr (WORD == W_F16) acc2.zero();
  gload(0);
  for (int t0 = 0; t0 < T; t0 += KS) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      int row = rq + 16 * q;
      uint32_t hh, ll;
      split_word<WORD>(ra[q].x * rw, ra[q].y * rw, sA, hh, ll);
      L.ahi[row * SW + kq] = hh;
      L.alo[row * SW + kq] = ll;
      split_word<WORD>(rb_[q].x, -rb_[q].y, sB, hh, ll);
      L.bhi[row * SW + kq] = hh;
      L.blo[row * SW + kq] = ll;
    }
    __syncthreads();
    if (t0 + KS < T) gload(t0 + KS);
    mma_stage16<WORD>(L, acc, acc2, wm, wn, lane);
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
          double re = acc.r[rb][cb][v], im = acc.i[rb][cb][v];
          if constexpr (WORD == W_F16) {
            re += (double)acc2.r[rb][cb][v] * (1.0 / 2048.0);
            im += (double)acc2.i[rb][cb][v] * (1.0 / 2048.0);
          }
          if constexpr (is_f16(WORD)) {
            re *= unscale;
            im *= unscale;
          }
          double2 p = Pj[(size_t)gi * N + gj];
          p.x += re;
          p.y += im;
          Pj[(size_t)gi * N + gj] = p;
        }
      }
    }
}

// FP16 path: weights as in weights_f32_kernel plus max |w_j| per frequency.
__global__ void weights_f32_max_kernel(const double* __restrict__ eps, int n_bands, int n_occ, Chunk c, OmegaList om,
                                       float* __restrict__ w, Scales* __restrict__ sc) {
  __shared__ float red[256];
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int T = c.T;
  double d = 0.0;
  if (t < T) {
    long g = c.tb + t;
    int n = c.n0 + (int)(g / c.nu);
    int u = c.u0 + (int)(g % c.nu);
    d = eps[(size_t)c.k * n_bands + n] - eps[(size_t)c.kq * n_bands + n_occ + u];
  }
  for (int j = 0; j < om.n; ++j) {
    float x = 0.f;
    if (t < T) {
      x = (float)pair_weight(d, om, j);
      w[(size_t)j * T + t] = x;
    }
    red[threadIdx.x] = fabsf(x);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) atomic_max_pos(&sc->w[j], red[0]);
    __syncthreads();
  }
}

// ------------------------------------------------------------ large-tile BF16
// 256 x 128 output tiles: 4 waves in a 2 x 2 arrangement, each owning 128 x 64
// complex outputs (4 x 2 blocks of 32 x 32, 256 FP32 accumulators per lane),
// LDS double-buffered so one barrier separates consecutive K stages.
constexpr int BM2 = 256, BN2 = 128;

struct Acc2 {
  floatx16 r[4][2];
  floatx16 i[4][2];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          r[a][b][v] = 0.f;
          i[a][b][v] = 0.f;
        }
  }
};

struct Lds2 {
  uint32_t ahi[BM2 * SW];
  uint32_t alo[BM2 * SW];
  uint32_t bhi[BN2 * SW];
  uint32_t blo[BN2 * SW];
};

__device__ inline void mma_stage_v2(const Lds2& L, Acc2& acc, int wm, int wn, int lane) {
  const int l32 = lane & 31, h = lane >> 5;
#pragma unroll
  for (int s = 0; s < KS / 8; ++s) {
    const int off = s * 8 + h * 4;
    uint4 brh[2], brl[2], bih[2], bil[2];
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
    for (int rb = 0; rb < 4; ++rb) {
      int row = wm * 128 + rb * 32 + l32;
      uint4 ah = *reinterpret_cast<const uint4*>(&L.ahi[row * SW + off]);
      uint4 al = *reinterpret_cast<const uint4*>(&L.alo[row * SW + off]);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc.r[rb][cb] = mma16<W_BF16>(ah, brh[cb], acc.r[rb][cb]);
        acc.i[rb][cb] = mma16<W_BF16>(ah, bih[cb], acc.i[rb][cb]);
        acc.r[rb][cb] = mma16<W_BF16>(ah, brl[cb], acc.r[rb][cb]);
        acc.i[rb][cb] = mma16<W_BF16>(ah, bil[cb], acc.i[rb][cb]);
        acc.r[rb][cb] = mma16<W_BF16>(al, brh[cb], acc.r[rb][cb]);
        acc.i[rb][cb] = mma16<W_BF16>(al, bih[cb], acc.i[rb][cb]);
      }
    }
  }
}

__device__ inline int acc2_row(int wm, int rb, int v, int lane) {
  return wm * 128 + rb * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

// Projection, BF16 words, 256 x 128 tiles, software-pipelined: the staging of
// stage s+1 (product, hi/lo split, LDS stores) is spread between the MFMA
// groups of stage s so that it issues in the shadow of the matrix cores, and
// global loads run one full stage ahead.  Loads are branch-free (addresses
// clamped inside the arrays, values zeroed by selects).
__global__ __launch_bounds__(NT, 1) void project_bf16_large_kernel(int N, int R, int Rp, const uint32_t* __restrict__ Uh,
                                                               const uint32_t* __restrict__ Ul,
                                                               const float2* __restrict__ po,
                                                               const float2* __restrict__ pu, int nu, long tb, int T,
                                                               float2* __restrict__ M, long ldm) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  Lds2* Lb = reinterpret_cast<Lds2*>(lds_raw);
  const int t0 = blockIdx.x * BN2;
  const int i0 = blockIdx.y * BM2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int l32 = lane & 31, h = lane >> 5;
  int aoff[4];
  uint32_t amask[4];
  size_t asrc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int e = tid + q * NT;
    int row = e >> 2, grp = e & 3;
    aoff[q] = row * SW + grp * 4;
    int gi = i0 + row;
    amask[q] = gi < N ? 0xffffffffu : 0u;
    asrc[q] = (size_t)(gi < N ? gi : 0) * Rp + grp * 4;
  }
  const int kq = tid % KS, rq = tid / KS;
  size_t ooff[LOADS], uoff[LOADS];
  float bmask[LOADS];
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    int gt = t0 + rq + 16 * q;
    bmask[q] = gt < T ? 1.f : 0.f;
    int t = gt < T ? gt : 0;
    const long g = tb + t;
    ooff[q] = (size_t)(g / nu) * R;
    uoff[q] = (size_t)(g % nu) * R;
  }
  uint4 rah[4], ral[4];
  float2 ro[LOADS], ru[LOADS];
  float rmask = 1.f;
  auto gload = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      rah[q] = *reinterpret_cast<const uint4*>(Uh + asrc[q] + r0);
      ral[q] = *reinterpret_cast<const uint4*>(Ul + asrc[q] + r0);
    }
    int r = r0 + kq;
    rmask = r < R ? 1.f : 0.f;
    r = r < R ? r : R - 1;
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      ro[q] = po[ooff[q] + r];
      ru[q] = pu[uoff[q] + r];
    }
  };
  auto store_a = [&](Lds2& L, int q) {
    uint4 x = rah[q], y = ral[q];
    x.x &= amask[q]; x.y &= amask[q]; x.z &= amask[q]; x.w &= amask[q];
    y.x &= amask[q]; y.y &= amask[q]; y.z &= amask[q]; y.w &= amask[q];
    *reinterpret_cast<uint4*>(&L.ahi[aoff[q]]) = x;
    *reinterpret_cast<uint4*>(&L.alo[aoff[q]]) = y;
  };
  auto store_b = [&](Lds2& L, int q) {
    const float m = bmask[q] * rmask;
    const int row = rq + 16 * q;
    float fr = (ro[q].x * ru[q].x + ro[q].y * ru[q].y) * m;
    float fi = (ro[q].x * ru[q].y - ro[q].y * ru[q].x) * m;
    uint32_t hh, ll;
    split_word<W_BF16>(fr, fi, 1.f, hh, ll);
    L.bhi[row * SW + kq] = hh;
    L.blo[row * SW + kq] = ll;
  };
  Acc2 acc;
  acc.zero();
  const int nst = (R + KS - 1) / KS;
  gload(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) store_a(Lb[0], q);
#pragma unroll
  for (int q = 0; q < LOADS; ++q) store_b(Lb[0], q);
  if (nst > 1) gload(KS);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const Lds2& L = Lb[st & 1];
    Lds2& Ln = Lb[(st + 1) & 1];
#pragma unroll
    for (int s = 0; s < KS / 8; ++s) {
      const int off = s * 8 + h * 4;
      uint4 brh[2], brl[2], bih[2], bil[2];
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
      for (int rb = 0; rb < 4; ++rb) {
        int row = wm * 128 + rb * 32 + l32;
        uint4 ah = *reinterpret_cast<const uint4*>(&L.ahi[row * SW + off]);
        uint4 al = *reinterpret_cast<const uint4*>(&L.alo[row * SW + off]);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          acc.r[rb][cb] = mma16<W_BF16>(ah, brh[cb], acc.r[rb][cb]);
          acc.i[rb][cb] = mma16<W_BF16>(ah, bih[cb], acc.i[rb][cb]);
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          acc.r[rb][cb] = mma16<W_BF16>(ah, brl[cb], acc.r[rb][cb]);
          acc.i[rb][cb] = mma16<W_BF16>(ah, bil[cb], acc.i[rb][cb]);
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          acc.r[rb][cb] = mma16<W_BF16>(al, brh[cb], acc.r[rb][cb]);
          acc.i[rb][cb] = mma16<W_BF16>(al, bih[cb], acc.i[rb][cb]);
        }
        // staging of the next stage, one slice per MFMA group (after the last
        // stage this writes the idle buffer, which is never read again)
        const int g = s * 4 + rb;
        if (g < 4) store_a(Ln, g);
        store_b(Ln, g);
        // 12 MFMAs interleaved with the slice's VALU and LDS work
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        }
      }
    }
    if (st + 2 < nst) gload((st + 2) * KS);
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      int gt = t0 + acc_col(wn, cb, lane);
      if (gt >= T) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int gi = i0 + acc2_row(wm, rb, v, lane);
        if (gi < N) M[(size_t)gi * ldm + gt] = make_float2(acc.r[rb][cb][v], acc.i[rb][cb][v]);
      }
    }
}

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

int launch_zero_u32(hipStream_t s, unsigned* p, int n) {
  hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  GW_LAUNCHED("zero_u32_kernel");
  return GW_OK;
}

int launch_maxabs(hipStream_t s, const float2* x, size_t n, unsigned* out) {
  unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(maxabs_kernel, dim3(std::max(1u, blocks)), dim3(256), 0, s, x, n, out);
  GW_LAUNCHED("maxabs_kernel");
  return GW_OK;
}

// Split U (and, for FP16, measure max|U| and max|psi| first).
int prepare_split(hipStream_t s, int word, int N, int R, int Rp, const float2* U, const float2* psi, size_t n_psi,
                  uint32_t* hi, uint32_t* lo, Scales* sc) {
  int st;
  if (word != W_BF16) {
    if ((st = launch_zero_u32(s, reinterpret_cast<unsigned*>(sc), (int)(sizeof(Scales) / 4))) != GW_OK) return st;
    if ((st = launch_maxabs(s, U, (size_t)N * R, &sc->u)) != GW_OK) return st;
    if ((st = launch_maxabs(s, psi, n_psi, &sc->psi)) != GW_OK) return st;
  }
  size_t n = (size_t)N * Rp;
  unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
  if (word == W_BF16)
    hipLaunchKernelGGL(split_u_kernel<W_BF16>, dim3(blocks), dim3(256), 0, s, N, R, Rp, U, sc, hi, lo);
  else if (word == W_F16)
    hipLaunchKernelGGL(split_u_kernel<W_F16>, dim3(blocks), dim3(256), 0, s, N, R, Rp, U, sc, hi, lo);
  else
    hipLaunchKernelGGL(split_u_kernel<W_F16S>, dim3(blocks), dim3(256), 0, s, N, R, Rp, U, sc, hi, lo);
  GW_LAUNCHED("split_u_kernel");
  return GW_OK;
}

// Large tiles pay off once the basis spans a few of them.
constexpr int kLargeTileN = 256;
int g_proj_variant = 2;   // 1: 128x128 tiles; 2: 256x128 software-pipelined (BF16 words only)
constexpr size_t kLds2Bytes = 2 * sizeof(Lds2);

int enable_large_lds() {
  static int done = 0;
  if (done) return GW_OK;
  GW_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&project_bf16_large_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds2Bytes));
  done = 1;
  return GW_OK;
}

int launch_herk16(hipStream_t s, int word, int N, int T, const float2* M, long ldm, const float* w, int n_omega,
                  double2* P, const Scales* sc) {
  const int ntile = (N + BM - 1) / BM;
  dim3 hgrid(ntile * (ntile + 1) / 2, n_omega);
  if (word == W_BF16) {
    ProfScope prof(s, "herk_bf16_kernel");
    hipLaunchKernelGGL(herk16_kernel<W_BF16>, hgrid, dim3(NT), 0, s, N, T, M, ldm, w, P, sc);
  } else if (word == W_F16) {
    ProfScope prof(s, "herk_f16_kernel");
    hipLaunchKernelGGL(herk16_kernel<W_F16>, hgrid, dim3(NT), 0, s, N, T, M, ldm, w, P, sc);
  } else {
    ProfScope prof(s, "herk_f16s_kernel");
    hipLaunchKernelGGL(herk16_kernel<W_F16S>, hgrid, dim3(NT), 0, s, N, T, M, ldm, w, P, sc);
  }
  GW_LAUNCHED("herk16_kernel");
  return GW_OK;
}

int launch_project16(hipStream_t s, int word, int N, int R, int Rp, const uint32_t* Uh, const uint32_t* Ul,
                     const float2* po, const float2* pu, int nu, long tb, int T, float2* M, long ldm, Scales* sc) {
  if (word == W_BF16 && g_proj_variant == 2 && N >= kLargeTileN) {
    int st = enable_large_lds();
    if (st != GW_OK) return st;
    dim3 grid2((T + BN2 - 1) / BN2, (N + BM2 - 1) / BM2);
    ProfScope prof(s, "project_bf16_kernel");
    hipLaunchKernelGGL(project_bf16_large_kernel, grid2, dim3(NT), kLds2Bytes, s, N, R, Rp, Uh, Ul, po, pu, nu, tb, T,
                       M, ldm);
    GW_LAUNCHED("project_bf16_large_kernel");
    return GW_OK;
  }
  dim3 grid((T + BN - 1) / BN, (N + BM - 1) / BM);
  if (word == W_BF16) {
    ProfScope prof(s, "project_bf16_kernel");
    hipLaunchKernelGGL(project16_kernel<W_BF16>, grid, dim3(NT), 0, s, N, R, Rp, Uh, Ul, po, pu, nu, tb, T, M, ldm, sc);
  } else if (word == W_F16) {
    ProfScope prof(s, "project_f16_kernel");
    hipLaunchKernelGGL(project16_kernel<W_F16>, grid, dim3(NT), 0, s, N, R, Rp, Uh, Ul, po, pu, nu, tb, T, M, ldm, sc);
  } else {
    ProfScope prof(s, "project_f16s_kernel");
    hipLaunchKernelGGL(project16_kernel<W_F16S>, grid, dim3(NT), 0, s, N, R, Rp, Uh, Ul, po, pu, nu, tb, T, M, ldm,
                       sc);
  }
  GW_LAUNCHED("project16_kernel");
  return GW_OK;
}

}  // namespace

// Pairs per chunk: a multiple of the 128-pair tile width, at most 8192 and
// with the c64 M chunk under 256 MB (it is re-read by the accumulation), chosen
// so that the projection's workgroups fill whole rounds of the 256 CUs.
int g_bf16_pipeline = 2;
int g_gemm_staging = 3;
int g_complex_product = 3;
int g_fp16_core = 1;
int g_gemm3m_pipeline = 6;
int g_gemm3m_lead = 4;
int g_real_core = 2;

static bool tiled_path(int precision) {
  return (precision == GW_SPLIT_BF16 && g_bf16_pipeline == 2) || (precision == GW_SPLIT_FP16 && g_fp16_core == 2);
}

int mfma_default_chunk_pairs(int N, int R, int n_omega, int precision) {
  if (tiled_path(precision)) return tiled_default_chunk_pairs(N, R, n_omega);
  const int tile_rows = (precision == GW_SPLIT_BF16 && g_proj_variant == 2 && N >= kLargeTileN) ? BM2 : BM;
  const long rows = (N + tile_rows - 1) / tile_rows;
  const long cap = std::max<long>(1, std::min<long>(64, (256L << 20) / ((long)N * 8 * BN)));
  long best_x = cap;
  double best_eff = -1.0;
  for (long x = cap; x >= std::min<long>(cap, 8); --x) {
    long w = rows * x;
    double eff = (double)w / (double)(((w + 255) / 256) * 256);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best_x = x;
    }
  }
  return (int)(best_x * BN);
}


static size_t split_u_bytes(int precision, int N, int R) {
  if (precision == GW_FP32) return 0;
  size_t Rp = (size_t)round_up(R, KS);
  return 2 * align_up((size_t)N * Rp * sizeof(uint32_t)) + align_up(sizeof(Scales));
}

size_t mfma_pol_workspace(int precision, int N, int R, int tc, int n_omega, size_t psi_rows) {
  if (tiled_path(precision)) return tiled_pol_workspace(N, R, tc, n_omega, psi_rows);
  return split_u_bytes(precision, N, R) + align_up((size_t)N * tc * sizeof(float2)) +
         align_up((size_t)n_omega * tc * sizeof(float));
}

size_t mfma_project_workspace(int precision, int N, int R, int n_occ, int n_unocc) {
  if (tiled_path(precision)) return tiled_project_workspace(N, R, n_occ, n_unocc);
  return split_u_bytes(precision, N, R);
}

static int word_of(int precision) {
  return precision == GW_SPLIT_FP16 ? W_F16 : (precision == GW_FP16 ? W_F16S : W_BF16);
}

int mfma_project(hipStream_t s, int precision, int N, int R, int n_occ, int n_unocc, const void* U,
                 const void* psi_occ, const void* psi_unocc, void* M, void* ws, size_t ws_bytes) {
  (void)ws_bytes;
  if (precision == GW_FP32)
    return launch_project_f32(s, N, R, static_cast<const float2*>(U), static_cast<const float2*>(psi_occ),
                              static_cast<const float2*>(psi_unocc), n_unocc, 0, n_occ * n_unocc,
                              static_cast<float2*>(M), (long)n_occ * n_unocc);
  if (precision == GW_SPLIT_BF16 && g_bf16_pipeline == 2)
    return tiled_project(s, N, R, n_occ, n_unocc, static_cast<const float2*>(U), static_cast<const float2*>(psi_occ),
                         static_cast<const float2*>(psi_unocc), static_cast<float2*>(M), ws);
  if (precision == GW_SPLIT_FP16 && g_fp16_core == 2)
    return tiled_project_f16(s, N, R, n_occ, n_unocc, static_cast<const float2*>(U),
                             static_cast<const float2*>(psi_occ), static_cast<const float2*>(psi_unocc),
                             static_cast<float2*>(M), ws);
  const int word = word_of(precision);
  const int Rp = round_up(R, KS);
  Carver cv(ws);
  uint32_t* Uh = cv.take<uint32_t>((size_t)N * Rp);
  uint32_t* Ul = cv.take<uint32_t>((size_t)N * Rp);
  Scales* sc = cv.take<Scales>(1);
  int st;
  if (word != W_BF16) {
    // psi_occ and psi_unocc are separate arrays: take the larger of their maxima
    if ((st = launch_zero_u32(s, reinterpret_cast<unsigned*>(sc), (int)(sizeof(Scales) / 4))) != GW_OK) return st;
    if ((st = launch_maxabs(s, static_cast<const float2*>(psi_occ), (size_t)n_occ * R, &sc->psi)) != GW_OK) return st;
    if ((st = launch_maxabs(s, static_cast<const float2*>(psi_unocc), (size_t)n_unocc * R, &sc->psi)) != GW_OK)
      return st;
    if ((st = launch_maxabs(s, static_cast<const float2*>(U), (size_t)N * R, &sc->u)) != GW_OK) return st;
    size_t n = (size_t)N * Rp;
    unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 16384);
    if (word == W_F16)
      hipLaunchKernelGGL(split_u_kernel<W_F16>, dim3(blocks), dim3(256), 0, s, N, R, Rp,
                         static_cast<const float2*>(U), sc, Uh, Ul);
    else
      hipLaunchKernelGGL(split_u_kernel<W_F16S>, dim3(blocks), dim3(256), 0, s, N, R, Rp,
                         static_cast<const float2*>(U), sc, Uh, Ul);
    GW_LAUNCHED("split_u_kernel");
  } else if ((st = prepare_split(s, word, N, R, Rp, static_cast<const float2*>(U), nullptr, 0, Uh, Ul, sc)) != GW_OK) {
    return st;
  }
  return launch_project16(s, word, N, R, Rp, Uh, Ul, static_cast<const float2*>(psi_occ),
                          static_cast<const float2*>(psi_unocc), n_unocc, 0, n_occ * n_unocc,
                          static_cast<float2*>(M), (long)n_occ * n_unocc, sc);
}

int mfma_polarization(hipStream_t s, const gw_pol_desc& d, const std::vector<Chunk>& chunks, int tc,
                      const OmegaList& om, void* ws) {
  if (d.precision == GW_SPLIT_BF16 && g_bf16_pipeline == 2) return tiled_polarization(s, d, chunks, tc, om, ws);
  if (d.precision == GW_SPLIT_FP16 && g_fp16_core == 2) return tiled_polarization_f16(s, d, chunks, tc, om, ws);
  Carver cv(ws);
  const int Rp = round_up(d.R, KS);
  uint32_t* Uh = nullptr;
  uint32_t* Ul = nullptr;
  Scales* sc = nullptr;
  const bool split = d.precision != GW_FP32;
  const int word = word_of(d.precision);
  if (split) {
    Uh = cv.take<uint32_t>((size_t)d.N * Rp);
    Ul = cv.take<uint32_t>((size_t)d.N * Rp);
    sc = cv.take<Scales>(1);
  }
  float2* M = cv.take<float2>((size_t)d.N * tc);
  float* w = cv.take<float>((size_t)d.n_omega * tc);
  const float2* U = static_cast<const float2*>(d.U);
  const float2* psi = static_cast<const float2*>(d.psi);
  const int nb = d.n_occ + d.n_unocc;
  const int ntile = (d.N + BM - 1) / BM;
  double2* P = reinterpret_cast<double2*>(d.P);
  int st;
  if (split && (st = prepare_split(s, word, d.N, d.R, Rp, U, psi, (size_t)d.n_k * nb * d.R, Uh, Ul, sc)) != GW_OK)
    return st;
  for (const Chunk& c : chunks) {
    const int T = c.pairs();
    if (word != W_BF16 && split) {
      // per-chunk maxima of |M| and |w_j|
      if ((st = launch_zero_u32(s, &sc->m, 1 + kMaxOmega)) != GW_OK) return st;
      hipLaunchKernelGGL(weights_f32_max_kernel, dim3((T + 255) / 256), dim3(256), 0, s, d.eps, nb, d.n_occ, c, om,
                         w, sc);
      GW_LAUNCHED("weights_f32_max_kernel");
    } else {
      hipLaunchKernelGGL(weights_f32_kernel, dim3((T + 255) / 256), dim3(256), 0, s, d.eps, nb, d.n_occ, c, om, w);
      GW_LAUNCHED("weights_f32_kernel");
    }
    const float2* po = psi + ((size_t)c.k * nb + c.n0) * d.R;
    const float2* pu = psi + ((size_t)c.kq * nb + d.n_occ + c.u0) * d.R;
    dim3 hgrid(ntile * (ntile + 1) / 2, d.n_omega);
    if (!split) {
      if ((st = launch_project_f32(s, d.N, d.R, U, po, pu, c.nu, c.tb, T, M, T)) != GW_OK) return st;
      ProfScope prof(s, "herk_f32_kernel");
      hipLaunchKernelGGL(herk_f32_kernel, hgrid, dim3(NT), 0, s, d.N, T, M, (long)T, w, P);
      GW_LAUNCHED("herk_f32_kernel");
    } else {
      if ((st = launch_project16(s, word, d.N, d.R, Rp, Uh, Ul, po, pu, c.nu, c.tb, T, M, T, sc)) != GW_OK)
        return st;
      if ((st = launch_herk16(s, word, d.N, T, M, (long)T, w, d.n_omega, P, sc)) != GW_OK) return st;
    }
  }
  return GW_OK;
}

}  // namespace gw

extern "C" int gw_get_tuning(const char* key, int* value) {
  if (!key || !value) return gw::fail(GW_ERR_INVALID_ARG, "gw_get_tuning: key and value are required");
  const std::string k(key);
  if (k == "projection_variant") *value = gw::g_proj_variant;
  else if (k == "gemm_staging") *value = gw::g_gemm_staging;
  else if (k == "bf16_pipeline") *value = gw::g_bf16_pipeline;
  else if (k == "complex_product") *value = gw::g_complex_product;
  else if (k == "fp16_core") *value = gw::g_fp16_core;
  else if (k == "gemm3m_pipeline") *value = gw::g_gemm3m_pipeline;
  else if (k == "gemm3m_lead") *value = gw::g_gemm3m_lead;
  else if (k == "real_core") *value = gw::g_real_core;
  else return gw::fail(GW_ERR_INVALID_ARG, std::string("gw_get_tuning: unknown key ") + key);
  return GW_OK;
}

extern "C" int gw_set_tuning(const char* key, int value) {
  if (!key) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: key is NULL");
  const std::string k(key);
  if (k == "projection_variant") {
    if (value < 1 || value > 2) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: projection_variant is 1 or 2");
    gw::g_proj_variant = value;
    return GW_OK;
  }
  if (k == "gemm_staging") {
    if (value < 1 || value > 4) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: gemm_staging is 1 to 4");
    gw::g_gemm_staging = value;
    return GW_OK;
  }
  if (k == "fp16_core") {
    if (value < 1 || value > 2) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: fp16_core is 1 or 2");
    gw::g_fp16_core = value;
    return GW_OK;
  }
  if (k == "real_core") {
    if (value < 1 || value > 2) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: real_core is 1 or 2");
    gw::g_real_core = value;
    return GW_OK;
  }
  if (k == "gemm3m_lead") {
    if (value < 3 || value > 5) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: gemm3m_lead is 3 to 5");
    gw::g_gemm3m_lead = value;
    return GW_OK;
  }
  if (k == "gemm3m_pipeline") {
    if (value != 2 && value != 6) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: gemm3m_pipeline is 2 or 6");
    gw::g_gemm3m_pipeline = value;
    return GW_OK;
  }
  if (k == "complex_product") {
    if (value != 3 && value != 4) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: complex_product is 3 or 4");
    gw::g_complex_product = value;
    return GW_OK;
  }
  if (k == "bf16_pipeline") {
    if (value < 1 || value > 2) return gw::fail(GW_ERR_INVALID_ARG, "gw_set_tuning: bf16_pipeline is 1 or 2");
    gw::g_bf16_pipeline = value;
    return GW_OK;
  }
  return gw::fail(GW_ERR_INVALID_ARG, std::string("gw_set_tuning: unknown key ") + key);
}
