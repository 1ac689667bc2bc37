// Fused block SRHT apply with the Hadamard factor H_16 on BF16 matrix cores
// ("split-BF16"): Y = Omega A (section 2, eq. (2.3)-(2.4)) for row-major A
// (n x m), the same result as the FP32 butterfly kernel up to rounding.
//
// Kronecker form (section 2): for a chunk of b = NW*BR rows of one block
// (NW = 8 waves, or 16 when l > 512 so that one thread serves each sample),
// H_b = H_NW (x) H_{BR/16} (x) H_16 over the bit fields of the chunk row
// x = BR*w' + 16*t_hi + x_16 (w' = wave).  Per chunk:
//   1. load  : lane (q, g) = (lane & 15, lane >> 4) fetches 16 bytes
//              (columns 4q .. 4q+3) of rows 4t + g, t in [0, BR/4): one
//              dwordx4 load per t covers 4 rows x 64 columns;
//   2. D^(i) : per-row sign flips (sign-bit xor; the row depends on g);
//   3. H_16  : one v_mfma_f32_16x16x32_bf16 per (t_hi, column e): the 32-long
//              K dimension holds [hi; lo] of the 16 rows x_16 = g + 4*t_lo,
//              against the operand [H_16 | H_16], so the product is
//              H_16 (hi + lo) accumulated in FP32.  hi = RNE_bf16(v),
//              lo = RNE_bf16(v - hi) (v - hi is exact in FP32), so
//              |v - hi - lo| <= 2^-16 |v|;
//   4. H_{BR/16} over t_hi in FP32 registers (applied before step 3: the
//      factors act on disjoint bit fields and commute), then LDS stores;
//   5. H_NW over the waves through LDS and the output-pruned gather of the
//      l sampled rows, as in the FP32 kernel:
//        (H_r v)[R_j] = sum_{x_hi} (-1)^popcount(R_j,hi & x_hi)
//                       * (H_b v_{x_hi})[R_j,lo].
// A is read exactly once; the sum over blocks (2.4) stays in registers; row
// splits write l x m partials summed in fixed order by the FP32 file's
// reduce.  As in the FP32 kernel, the 16-wave instance writes the
// exchange's output to a second LDS buffer read by the gather, which removes
// the barrier between the gather and the next chunk's stores.  Blocks shorter than 128 rows (r < 128) have no room for an H_16
// tile per wave and are computed by the FP32 kernels.
#include <limits.h>

#include "common.h"

namespace bsrht {
namespace {

constexpr int kCT = 64;         // columns per workgroup
constexpr int kLDT = kCT + 4;   // LDS row stride in floats
constexpr int kBufDword3 = 0x00020000;  // raw buffer resource word 3 (gfx9 family)
constexpr int kAuxNT = 2;       // non-temporal loads (A is read once)

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

struct Bf16Args {
  const float *A;
  int64_t lda;
  int m;
  const int32_t *R;
  const uint32_t *Dbits;
  const uint32_t *Dtbits;
  int dt_words;
  int l;
  int log2r;
  int chunks_per_split;
  int total_chunks;
  int tile0;  // first column tile of this launch
  float *out;
  int64_t ldo;
  int64_t split_stride;
  float scale;
  const int32_t *order;  // sample of each gather lane
};

// hi/lo BF16 split of two values, packed two per dword (first value low).
__device__ __forceinline__ void split_pair(float a, float b, uint32_t &hi, uint32_t &lo) {
  const bf16x2_t h = __builtin_convertvector((float2_t){a, b}, bf16x2_t);
  hi = __builtin_bit_cast(uint32_t, h);
  const float ha = __uint_as_float(hi << 16), hb = __uint_as_float(hi & 0xffff0000u);
  const bf16x2_t lw = __builtin_convertvector((float2_t){a - ha, b - hb}, bf16x2_t);
  lo = __builtin_bit_cast(uint32_t, lw);
}

// Two entries H_16[r][x0], H_16[r][x1] as packed BF16 (+-1 is exact).
__device__ __forceinline__ uint32_t h16_pair(int r, int x0, int x1) {
  const uint32_t s0 = (uint32_t)__popc(r & x0) & 1u, s1 = (uint32_t)__popc(r & x1) & 1u;
  return (0x3F80u | (s0 << 15)) | ((0x3F80u | (s1 << 15)) << 16);
}

template <int N>
__device__ __forceinline__ void fwht_regs(float (&v)[N]) {
#pragma unroll
  for (int h = 1; h < N; h <<= 1) {
#pragma unroll
    for (int x = 0; x < N; ++x) {
      if ((x & h) == 0) {
        const float a = v[x], b = v[x + h];
        v[x] = a + b;
        v[x + h] = a - b;
      }
    }
  }
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, -1, kBufDword3);
}

template <int NW, int BR, bool RAGGED>
struct Bf16Cta {
  static constexpr int B = BR * NW;
  static constexpr int LOG2B = ilog2c(B);
  static constexpr int NT = BR / 4;   // row quads per wave
  static constexpr int NH = NT / 4;   // values of t_hi
  static constexpr int G = BR / NW;  // H_NW groups per wave
  static_assert(BR >= 16 && BR <= 64, "BR in {16, 32, 64}");

  float *T;
  float *T2 = nullptr;  // second buffer: exchange output, gather input
  const Bf16Args &a;
  int lane, w, q4, g, j, pos, cpb_log2, row_bytes;
  int voff[RAGGED ? 4 : 1];  // byte offset of the lane's columns in its row 4t+g
  bool jok;
  uint32_t rhi;
  int cur_block;
  uint32_t dtbit;
  const u32x4_t *hop_lds;     // this lane's [H_16 | H_16] operand in LDS
  const float *wavebase;      // A + c0 + w*BR*lda (wave-uniform)
  float acc[kCT];

  __device__ __forceinline__ Bf16Cta(float *T_, const Bf16Args &a_) : T(T_), a(a_) {}

  __device__ __forceinline__ const float *chunk_base(int q) const {
    return wavebase + (int64_t)q * B * a.lda;
  }

  template <int T0, int T1>
  __device__ __forceinline__ void load(float4 (&v)[NT], const float *base) const {
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(base);
#pragma unroll
    for (int t = T0; t < T1; ++t) {
      const int soff = 4 * t * row_bytes;
      if constexpr (RAGGED) {
        v[t].x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff[0], soff, kAuxNT));
        v[t].y = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff[1], soff, kAuxNT));
        v[t].z = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff[2], soff, kAuxNT));
        v[t].w = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff[3], soff, kAuxNT));
      } else {
        const u32x4_t u = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[0], soff, kAuxNT);
        v[t] = make_float4(__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z),
                           __uint_as_float(u.w));
      }
    }
  }

  // D^(i) for the wave's rows g0 + 4t + g (g0 = global row of the wave's
  // first row, a multiple of BR).
  __device__ __forceinline__ void dsigns(float4 (&v)[NT], int64_t g0) const {
    uint32_t wl[BR >= 32 ? BR / 32 : 1];
    if constexpr (BR >= 32) {
#pragma unroll
      for (int k = 0; k < BR / 32; ++k) wl[k] = a.Dbits[(g0 >> 5) + k] >> g;
    } else {
      wl[0] = (a.Dbits[g0 >> 5] >> (uint32_t)(g0 & 31)) >> g;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const uint32_t msk = (wl[t >> 3] << (31 - 4 * (t & 7))) & 0x80000000u;
      v[t].x = __uint_as_float(__float_as_uint(v[t].x) ^ msk);
      v[t].y = __uint_as_float(__float_as_uint(v[t].y) ^ msk);
      v[t].z = __uint_as_float(__float_as_uint(v[t].z) ^ msk);
      v[t].w = __uint_as_float(__float_as_uint(v[t].w) ^ msk);
    }
  }

  // H over t_hi in FP32 registers, in place.  (Transforms over disjoint bit
  // fields commute, so applying it before H_16 does not change the result.)
  __device__ __forceinline__ void h_thi(float4 (&v)[NT]) const {
    if constexpr (NH > 1) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        float u[4][NH];
#pragma unroll
        for (int th = 0; th < NH; ++th) {
          u[0][th] = v[4 * th + s].x;
          u[1][th] = v[4 * th + s].y;
          u[2][th] = v[4 * th + s].z;
          u[3][th] = v[4 * th + s].w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) fwht_regs<NH>(u[e]);
#pragma unroll
        for (int th = 0; th < NH; ++th)
          v[4 * th + s] = make_float4(u[0][th], u[1][th], u[2][th], u[3][th]);
      }
    }
  }

  // H_16 on the matrix cores for t_hi in [TH0, TH1); the results go to LDS
  // rows w*BR + 16*t_hi + 4g + v, columns 4q .. 4q+3.
  template <int TH0, int TH1>
  __device__ __forceinline__ void mfma_store(const float4 (&v)[NT]) {
    // Re-read per chunk rather than held: registers are tightest in the
    // gather, where this operand is not needed.
    const bf16x8_t hop = __builtin_bit_cast(bf16x8_t, *hop_lds);
#pragma unroll
    for (int th = TH0; th < TH1; ++th) {
      floatx4_t d[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float4 &f = v[4 * th + s];
          x[s] = e == 0 ? f.x : e == 1 ? f.y : e == 2 ? f.z : f.w;
        }
        uint32_t h01, l01, h23, l23;
        split_pair(x[0], x[1], h01, l01);
        split_pair(x[2], x[3], h23, l23);
        const bf16x8_t bop = __builtin_bit_cast(bf16x8_t, (u32x4_t){h01, h23, l01, l23});
        const floatx4_t zero = {0.f, 0.f, 0.f, 0.f};
        d[e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hop, bop, zero, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float4 *dst =
            reinterpret_cast<float4 *>(T + (w * BR + 16 * th + 4 * g + r) * kLDT + 4 * q4);
        *dst = make_float4(d[0][r], d[1][r], d[2][r], d[3][r]);
      }
    }
  }

  __device__ __forceinline__ void step(int q, int q1, float4 (&cur)[NT], float4 (&nxt)[NT]) {
    // The next chunk is prefetched in two halves; the second is issued once
    // this chunk has left the registers for LDS, which keeps the
    // accumulators, one chunk and half a chunk within 256 VGPRs.
    const bool more = q + 1 < q1;
    if (more) load<0, NT / 2>(nxt, chunk_base(q + 1));
    dsigns(cur, (int64_t)q * B + w * BR);
    h_thi(cur);
    mfma_store<0, NH>(cur);
    if (more) load<NT / 2, NT>(nxt, chunk_base(q + 1));
    __syncthreads();
    // H_NW over the waves: group t holds rows t, t+BR, ..., t+(NW-1)*BR.
    float *const Tx = T2 ? T2 : T;  // where the exchange writes and the gather reads
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      const float *Tg = T + (w * G + gi) * kLDT + lane;
      float *Og = Tx + (w * G + gi) * kLDT + lane;
      float u[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) u[k] = Tg[k * BR * kLDT];
      fwht_regs<NW>(u);
#pragma unroll
      for (int k = 0; k < NW; ++k) Og[k * BR * kLDT] = u[k];
    }
    __syncthreads();
    if (jok) {
      const int i = q >> cpb_log2;
      if (i != cur_block) {
        cur_block = i;
        dtbit = (a.Dtbits[(int64_t)i * a.dt_words + (j >> 5)] >> (j & 31)) & 1u;
      }
      const uint32_t xhi = (uint32_t)q & ((1u << cpb_log2) - 1u);
      const uint32_t par = (uint32_t)__popc(rhi & xhi) & 1u;
      const float sgn = (par ^ dtbit) ? -1.f : 1.f;
      const float4 *row = reinterpret_cast<const float4 *>(Tx + pos * kLDT);
#pragma unroll
      for (int c4 = 0; c4 < kCT / 4; ++c4) {
        const float4 u = row[c4];
        acc[4 * c4 + 0] = fmaf(sgn, u.x, acc[4 * c4 + 0]);
        acc[4 * c4 + 1] = fmaf(sgn, u.y, acc[4 * c4 + 1]);
        acc[4 * c4 + 2] = fmaf(sgn, u.z, acc[4 * c4 + 2]);
        acc[4 * c4 + 3] = fmaf(sgn, u.w, acc[4 * c4 + 3]);
      }
    }
    // With two buffers the next exchange writes T2 only after the next
    // chunk's first barrier, which every wave passes after this gather.
    if (!T2) __syncthreads();
  }
};

template <int NW, int BR, bool RAGGED>
__global__ __launch_bounds__(NW * 64) void fused_bf16_kernel(Bf16Args a) {
  using Cta = Bf16Cta<NW, BR, RAGGED>;
  constexpr bool DB = NW == 16;  // two LDS buffers (see the file comment)
  __shared__ __attribute__((aligned(16))) float T[(DB ? 2 : 1) * Cta::B * kLDT];
  __shared__ u32x4_t Hop[64];
  Cta cta(T, a);
  cta.T2 = DB ? T + Cta::B * kLDT : nullptr;
  const int tid = threadIdx.x;
  cta.lane = tid & 63;
  cta.w = __builtin_amdgcn_readfirstlane(tid >> 6);
  cta.q4 = cta.lane & 15;
  cta.g = cta.lane >> 4;
  int bx = blockIdx.x, by = blockIdx.y;
  {
    const int nwg = (int)(gridDim.x * gridDim.y);
    if ((nwg & 7) == 0) {
      const int lin = (int)(blockIdx.x + gridDim.x * blockIdx.y);
      const int idx = (lin & 7) * (nwg >> 3) + (lin >> 3);
      bx = idx % (int)gridDim.x;
      by = idx / (int)gridDim.x;
    }
  }
  const int c0 = (a.tile0 + bx) * kCT;
  cta.row_bytes = (int)(a.lda * 4);
  if constexpr (RAGGED) {
    // Columns past m load a valid neighbour (column m-1); they never reach Y.
#pragma unroll
    for (int e = 0; e < 4; ++e)
      cta.voff[e] = (min(c0 + 4 * cta.q4 + e, a.m - 1) - c0) * 4 + cta.g * cta.row_bytes;
  } else {
    cta.voff[0] = 16 * cta.q4 + cta.g * cta.row_bytes;
  }
  cta.wavebase = a.A + c0 + (int64_t)(cta.w * BR) * a.lda;
  // [H_16 | H_16] operand: lane (r, g) holds H_16[r][g + 4s], s = 0..3, for
  // the hi half of K and again for the lo half.
  if (tid < 64) {
    const int r = tid & 15, gg = tid >> 4;
    const uint32_t h01 = h16_pair(r, gg, gg + 4), h23 = h16_pair(r, gg + 8, gg + 12);
    Hop[tid] = (u32x4_t){h01, h23, h01, h23};
  }
  cta.hop_lds = &Hop[cta.lane];
  __syncthreads();
  const int q0 = by * a.chunks_per_split;
  const int q1 = min(q0 + a.chunks_per_split, a.total_chunks);
  // Lanes take the samples in the plan's bank-spreading order, as in the
  // FP32 kernel.
  const int lidx = blockIdx.z * (NW * 64) + tid;
  cta.jok = lidx < a.l;
  cta.j = cta.jok ? a.order[lidx] : lidx;
  const int rj = cta.jok ? a.R[cta.j] : 0;
  cta.pos = rj & (Cta::B - 1);
  cta.rhi = (uint32_t)rj >> Cta::LOG2B;
  cta.cpb_log2 = a.log2r - Cta::LOG2B;
  cta.cur_block = -1;
  cta.dtbit = 0;
#pragma unroll
  for (int k = 0; k < kCT; ++k) cta.acc[k] = 0.f;

  // One step per iteration and an explicit copy of the prefetched chunk (two
  // alternating step bodies made the register allocator spill into the
  // gather, where a reload waits for the whole prefetch).
  float4 bufA[Cta::NT], bufB[Cta::NT];
  if (q0 < q1) cta.template load<0, Cta::NT>(bufA, cta.chunk_base(q0));
#pragma nounroll
  for (int q = q0; q < q1; ++q) {
    cta.step(q, q1, bufA, bufB);
#pragma unroll
    for (int t = 0; t < Cta::NT; ++t) bufA[t] = bufB[t];
  }

  if (cta.jok) {
    float *o = a.out + (int64_t)by * a.split_stride + (int64_t)cta.j * a.ldo + c0;
    const int ncol = min(kCT, a.m - c0);
#pragma unroll
    for (int k = 0; k < kCT; ++k)
      if (k < ncol) o[k] = cta.acc[k] * a.scale;
  }
}

struct Launch {
  bool fp32 = false;
  int nw = 8, br = 0, b = 0;
  int full_tiles = 0, ragged = 0, groups = 0, splits = 1, cps = 0, total_chunks = 0;
  size_t ws = 0;
};

Launch choose_launch(const bsrht_plan_s *pl, int64_t m) {
  Launch L;
  int per_cu;
  if (pl->r != pl->rp) {  // blocks padded with zeros: the FP32 kernels
    L.fp32 = true;
    return L;
  }
  if (pl->l > 512 && pl->r >= 256) {
    // 16 waves, one thread per sample for l <= 1024: A is read once per
    // 1024 samples; chunks of b = 16*16 rows.
    L.nw = 16;
    L.br = 16;
    per_cu = 1;
  } else {
    // Largest chunk b = 8*BR <= r with 16 <= BR <= 64.
    int br = 64;
    while (br >= 16 && (int64_t)br * 8 > pl->r) br >>= 1;
    if (br < 16) {
      L.fp32 = true;
      return L;
    }
    L.nw = 8;
    L.br = br;
    per_cu = br * 8 * kLDT * 4 > 80 * 1024 ? 1 : 2;
  }
  L.b = L.br * L.nw;
  L.total_chunks = (int)(pl->n / L.b);
  L.full_tiles = (int)(m / kCT);
  L.ragged = (m % kCT) != 0 ? 1 : 0;
  const int ctiles = L.full_tiles + L.ragged;
  const int spp = L.nw * 64;
  L.groups = (int)((pl->l + spp - 1) / spp);
  const int64_t target = (int64_t)device_cu_count() * per_cu;
  int64_t splits = target / ((int64_t)ctiles * L.groups);
  if (splits < 1) splits = 1;
  if (splits > L.total_chunks) splits = L.total_chunks;
  L.cps = (int)((L.total_chunks + splits - 1) / splits);
  L.splits = (L.total_chunks + L.cps - 1) / L.cps;
  L.ws = L.splits > 1 ? (size_t)L.splits * (size_t)pl->l * (size_t)m * sizeof(float) : 0;
  return L;
}

template <int NW, int BR>
int launch_bf16(const Launch &L, Bf16Args &a, hipStream_t s) {
  const int tslot = timing_begin(BSRHT_TIMING_APPLY_BF16, s);
  if (L.full_tiles > 0) {
    a.tile0 = 0;
    dim3 grid((unsigned)L.full_tiles, (unsigned)L.splits, (unsigned)L.groups);
    fused_bf16_kernel<NW, BR, false><<<grid, NW * 64, 0, s>>>(a);
  }
  if (L.ragged) {
    a.tile0 = L.full_tiles;
    dim3 grid(1u, (unsigned)L.splits, (unsigned)L.groups);
    fused_bf16_kernel<NW, BR, true><<<grid, NW * 64, 0, s>>>(a);
  }
  timing_end(tslot, s);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

}  // namespace

size_t apply_split_bf16_ws_bytes(const bsrht_plan_s *pl, int64_t m) {
  if (!pl || m <= 0) return 0;
  const Launch L = choose_launch(pl, m);
  if (L.fp32) return apply_fp32_ws_bytes(pl, m);
  return L.ws;
}

int apply_split_bf16(const bsrht_plan_s *pl, const float *A, int64_t m, int64_t lda, float *Y,
                     int64_t ldy, void *ws, size_t ws_bytes, hipStream_t s) {
  const Launch L = choose_launch(pl, m);
  if (L.fp32) return apply_fp32(pl, A, m, lda, Y, ldy, ws, ws_bytes, s);
  if (L.groups > 65535) return BSRHT_EUNSUPPORTED;
  // Row offsets inside one wave's BR rows are 32-bit buffer offsets.
  if ((int64_t)L.br * lda * 4 >= (int64_t(1) << 31)) return BSRHT_EUNSUPPORTED;
  if (ws_bytes < L.ws || (L.ws && !ws)) return BSRHT_ENOMEM;
  const float scale = 1.0f / sqrtf((float)pl->l);
  Bf16Args a;
  a.A = A;
  a.lda = lda;
  a.m = (int)m;
  a.R = pl->R;
  a.order = pl->order;
  a.Dbits = pl->Dbits;
  a.Dtbits = pl->Dtbits;
  a.dt_words = (int)pl->dt_words;
  a.l = (int)pl->l;
  a.log2r = pl->log2r;
  a.chunks_per_split = L.cps;
  a.total_chunks = L.total_chunks;
  a.tile0 = 0;
  if (L.splits > 1) {
    a.out = static_cast<float *>(ws);
    a.ldo = m;
    a.split_stride = pl->l * m;
    a.scale = 1.0f;
  } else {
    a.out = Y;
    a.ldo = ldy;
    a.split_stride = 0;
    a.scale = scale;
  }
  int st;
  if (L.nw == 16) {
    st = launch_bf16<16, 16>(L, a, s);
  } else {
    switch (L.br) {
      case 64: st = launch_bf16<8, 64>(L, a, s); break;
      case 32: st = launch_bf16<8, 32>(L, a, s); break;
      default: st = launch_bf16<8, 16>(L, a, s); break;
    }
  }
  if (st != BSRHT_OK) return st;
  if (L.splits > 1)
    return reduce_splits(static_cast<const float *>(ws), L.splits, pl->l * m, pl->l, m, Y, ldy,
                         scale, s);
  return BSRHT_OK;
}

}  // namespace bsrht
