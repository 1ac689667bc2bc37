// Block SRHT applied from the right, FP32 butterflies: Y = A Omega^T for a
// row-major A (m x n), the orientation of Algorithm 1 (section 3.1), where
// each row of A is sketched along its contiguous dimension.  For row g with
// block segments a_g^(i) (r consecutive entries each), eq. (2.3)-(2.4) give
//   Y[g, j] = (1/sqrt(l)) sum_i Dt^(i)_j (H_r D^(i) a_g^(i))[R_j].
//
// Structure.  H_r factors as H_{r/b} (x) H_b for the split x = x_hi*b + x_lo
// (Kronecker form of H, section 2), and H_b itself factors over any grouping
// of the bits of x_lo.  A workgroup of NW waves owns 64 rows and streams
// chunks of b = 64*NW consecutive columns (one chunk = one x_hi of one block).
//   1. load  : 16-byte non-temporal loads, each wave instruction reading 256
//              consecutive floats of one row; the next chunk is in flight.
//              Thread (w, lane) holds rows w*RW + s (RW = 64/NW) at columns
//              x = k*256 + 4*lane + c  (k < b/256, c < 4);
//   2. D^(i) : per-column sign flips (sign-bit xor);
//   3. H over the x bits each thread holds (bits 0, 1 and 8 .. log2 b - 1),
//              in registers;
//   4. LDS   : the chunk is stored as T[x][row] (rows contiguous, groups of
//              four rows XOR-swizzled by x bits 2..5, which makes the stores
//              and the reads of step 4 conflict-free); each thread then reads
//              the 64 values of one (row, x bits 0, 1, 8..) over x bits 2..7,
//              applies H_64 in registers and stores them back: the chunk now
//              holds H_b of every row's segment;
//   5. gather: thread = sample j adds +-T[R_j mod b][0..63] to its 64 row
//              accumulators, with sign Dt^(i)_j (-1)^popcount(R_j,hi & x_hi).
// The accumulators run across chunks and blocks (the sum (2.4) happens in
// registers); A is read once.  Column splits (for parallelism) write m x l
// partials that a second kernel sums in fixed split order and scales by
// 1/sqrt(l).  Blocks shorter than 256 columns use a direct evaluation.
//
// Padded blocks (section 2's partial SRHT: r < 2^log2r, each block of A
// treated as r columns and zeros): the launch walks only the chunks that
// hold columns of A (ceil(r / b) per block), each at column i*r + x_hi*b of
// A, with its signs, H_{r/b} factor and Dt block taken at its place in the
// padded layout; the last chunk of a block loads its columns past r as
// zeros (addresses clamped into the block, values masked).
#include <limits.h>

#include "common.h"

namespace bsrht {
namespace {

constexpr int kRT = 64;  // rows per workgroup tile (one accumulator per row)
constexpr int kBufDword3 = 0x00020000;  // raw buffer resource word 3 (gfx9 family)
constexpr int kAuxNT = 2;               // buffer cache policy: non-temporal
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, kBufDword3);
}

struct RightArgs {
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
  float *out;
  int64_t ldo;
  int64_t split_stride;
  float scale;
  const int32_t *order;  // sample of each gather lane
  // PAD plans (r < 2^log2r): the blocks hold r columns of A each and are
  // padded with zeros; chunk qr of the launch's chunks is chunk qr mod cr of
  // block qr / cr, and chunks past a block's r columns are skipped.
  int64_t r_cols;
  int cr;  // chunks per block that hold columns of A
};

// Unscaled Walsh-Hadamard transform of N values held in registers.
template <int N>
__device__ __forceinline__ void fwht64_regs(float (&v)[N]) {
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

// H over the register index kc (x bits 0, 1 and 8..) for each of the RW rows;
// v[kc*RW + s] holds row s at register index kc.
template <int NK, int RW>
__device__ __forceinline__ void fwht_kc(float (&v)[NK * RW]) {
#pragma unroll
  for (int h = 1; h < NK; h <<= 1) {
#pragma unroll
    for (int kc = 0; kc < NK; ++kc) {
      if ((kc & h) == 0) {
#pragma unroll
        for (int s = 0; s < RW; ++s) {
          const float a = v[kc * RW + s], b = v[(kc + h) * RW + s];
          v[kc * RW + s] = a + b;
          v[(kc + h) * RW + s] = a - b;
        }
      }
    }
  }
}

// LDS offset (floats) of row group g4 (rows 4*g4 .. 4*g4+3) at chunk column x.
__device__ __forceinline__ int tofs(int x, int g4) {
  return x * kRT + 4 * (g4 ^ ((x >> 2) & 15));
}

template <int NW, bool PAD = false>
struct RightCta {
  static constexpr int B = 64 * NW;      // chunk columns
  static constexpr int LOG2B = 6 + (NW == 8 ? 3 : 2);
  static constexpr int K = B / 256;      // 256-column slices per row
  static constexpr int NK = 4 * K;       // register indices per row
  static constexpr int RW = kRT / NW;    // rows per wave
  static_assert(NK * RW == 64, "64 values per thread");
  static_assert(NK == NW, "one wave per register index in step 4");

  float *T;
  const RightArgs &a;
  int lane, w, j, jc, pos, swz, cpb_log2;
  bool jok;
  uint32_t rhi;  // R_j's chunk-index bits (R_j >> log2 b)
  const float *wavebase;  // A + (first row of this wave) * lda (wave-uniform)
  int rowoff[RW];         // byte offsets of the wave's rows from wavebase (uniform)
  float acc[kRT];  // one per row of the tile

  __device__ __forceinline__ RightCta(float *T_, const RightArgs &a_) : T(T_), a(a_) {}

  // Chunk q of the launch in the padded layout: its index qp among all
  // 2^log2r / b chunks of the blocks (which the signs and H_{r/b} use), the
  // column of A where it starts and how many of its columns hold data.
  __device__ __forceinline__ void locate(int q, int &qp, int64_t &xa, int &vr) const {
    if constexpr (PAD) {
      const int i = __builtin_amdgcn_readfirstlane(q / a.cr);
      const int xh = q - i * a.cr;
      qp = (i << cpb_log2) + xh;
      xa = (int64_t)i * a.r_cols + (int64_t)xh * B;
      const int64_t rem = a.r_cols - (int64_t)xh * B;
      vr = rem < B ? (int)rem : B;
    } else {
      qp = q;
      xa = (int64_t)q * B;
      vr = B;
    }
  }

  // Loads chunk q into v, its D^(i) words into d and the Dt^(i) word of
  // sample j into dt (raw words: decoding them here would make the wave wait
  // for the loads just issued).
  __device__ __forceinline__ void load(float (&v)[64], uint32_t (&d)[K + 1], int q) const {
    int qp, vr;
    int64_t xa;
    locate(q, qp, xa, vr);
    const int64_t x0 = (int64_t)qp * B;  // the chunk's first column in the padded layout
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(wavebase + xa);
    const int voff = lane * 16;
    if (!PAD || vr == B) {
#pragma unroll
      for (int s = 0; s < RW; ++s) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const i32x4 t = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 1024 * k, rowoff[s], kAuxNT);
          v[(4 * k + 0) * RW + s] = __int_as_float(t.x);
          v[(4 * k + 1) * RW + s] = __int_as_float(t.y);
          v[(4 * k + 2) * RW + s] = __int_as_float(t.z);
          v[(4 * k + 3) * RW + s] = __int_as_float(t.w);
        }
      }
    } else {
      // the block's last chunk with data: columns past r are the padding.
      // Each value is loaded from a column clamped into the block's data
      // (so every address lies in A) and masked to zero past r.
#pragma unroll
      for (int s = 0; s < RW; ++s) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int x = 256 * k + 4 * lane + c;
            const int xc = x < vr ? x : vr - 1;
            const uint32_t u = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, 4 * xc, rowoff[s], kAuxNT);
            v[(4 * k + c) * RW + s] = __uint_as_float(x < vr ? u : 0u);
          }
        }
      }
    }
    // D^(i) words of this lane's columns: column x0 + k*256 + 4*lane + c is
    // bit 4*(lane & 7) + c of word (x0 + k*256)/32 + lane/8.
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(a.Dbits + (x0 >> 5));
#pragma unroll
    for (int k = 0; k < K; ++k)
      d[k] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rd, (lane >> 3) * 4 + 32 * k, 0, 0);
    d[K] = a.Dtbits[(int64_t)(qp >> cpb_log2) * a.dt_words + (jc >> 5)];
  }

  // One chunk; with PREFETCH the next chunk's loads are issued first.
  template <bool PREFETCH>
  __device__ __forceinline__ void step(int q, float (&cur)[64], uint32_t (&dcur)[K + 1],
                                       float (&nxt)[64], uint32_t (&dnxt)[K + 1]) {
    if constexpr (PREFETCH) load(nxt, dnxt, q + 1);
    // D^(i): the sign of column x applies to every row.
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t dk = dcur[k] >> (4 * (lane & 7));
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t msk = (dk << (31 - c)) & 0x80000000u;
#pragma unroll
        for (int s = 0; s < RW; ++s) {
          float &x = cur[(4 * k + c) * RW + s];
          x = __uint_as_float(__float_as_uint(x) ^ msk);
        }
      }
    }
    fwht_kc<NK, RW>(cur);
    // Store T[x][row]: four consecutive rows per 16-byte store.
#pragma unroll
    for (int kc = 0; kc < NK; ++kc) {
      const int x = (kc >> 2) * 256 + 4 * lane + (kc & 3);
#pragma unroll
      for (int s4 = 0; s4 < RW / 4; ++s4) {
        float4 v4;
        v4.x = cur[kc * RW + 4 * s4 + 0];
        v4.y = cur[kc * RW + 4 * s4 + 1];
        v4.z = cur[kc * RW + 4 * s4 + 2];
        v4.w = cur[kc * RW + 4 * s4 + 3];
        *reinterpret_cast<float4 *>(T + tofs(x, w * (RW / 4) + s4)) = v4;
      }
    }
    __syncthreads();
    // H_64 over x bits 2..7: thread (w, lane) takes row = lane at register
    // index kc = w, i.e. columns x = (w >> 2)*256 + (w & 3) + 4*t, t < 64,
    // whose swizzled offset tofs(x, lane >> 2) + (lane & 3) reduces to
    // 64*x + (lane ^ 4*(t & 15)).  The empty asm keeps these 16 per-lane
    // offsets inside the loop (hoisted, they would occupy 16 registers for
    // the whole kernel).
    {
      int ln = lane;
      asm volatile("" : "+v"(ln));
      float *Tb = T + 64 * ((w >> 2) * 256 + (w & 3));
      float v[64];
#pragma unroll
      for (int t = 0; t < 64; ++t) v[t] = Tb[256 * t + (ln ^ (4 * (t & 15)))];
      fwht64_regs<64>(v);
#pragma unroll
      for (int t = 0; t < 64; ++t) Tb[256 * t + (ln ^ (4 * (t & 15)))] = v[t];
    }
    __syncthreads();
    if (jok) {
      const uint32_t dtbit = (dcur[K] >> (j & 31)) & 1u;
      int qp, vr;
      int64_t xa;
      locate(q, qp, xa, vr);
      const uint32_t xhi = (uint32_t)qp & ((1u << cpb_log2) - 1u);
      const uint32_t par = (uint32_t)__popc(rhi & xhi) & 1u;
      const float sgn = (par ^ dtbit) ? -1.f : 1.f;
      // Rows 4g .. 4g+3 of chunk column pos sit at float offset
      // 64*pos + 4*(g ^ swz) = a0 ^ 4g with a0 = 64*pos + 4*swz: one xor per
      // read, and lanes with different pos read different bank groups.  The
      // empty asm keeps the 16 offsets inside the loop.
      int a0 = pos * kRT + 4 * swz;
      asm volatile("" : "+v"(a0));
      // All 16 reads are issued before the accumulation (the registers of
      // the chunk just stored are free here), so their latencies overlap.
      float4 gv[kRT / 4];
#pragma unroll
      for (int g = 0; g < kRT / 4; ++g)
        gv[g] = *reinterpret_cast<const float4 *>(T + (a0 ^ (4 * g)));
#pragma unroll
      for (int g = 0; g < kRT / 4; ++g) {
        acc[4 * g + 0] = fmaf(sgn, gv[g].x, acc[4 * g + 0]);
        acc[4 * g + 1] = fmaf(sgn, gv[g].y, acc[4 * g + 1]);
        acc[4 * g + 2] = fmaf(sgn, gv[g].z, acc[4 * g + 2]);
        acc[4 * g + 3] = fmaf(sgn, gv[g].w, acc[4 * g + 3]);
      }
    }
    __syncthreads();
  }
};

template <int NW, bool PAD = false>
__global__ __launch_bounds__(NW * 64) void right_fp32_kernel(RightArgs a) {
  using Cta = RightCta<NW, PAD>;
  __shared__ __attribute__((aligned(16))) float T[Cta::B * kRT];
  // XCD-aware tile order (workgroup k runs on XCD k mod 8): each XCD gets a
  // contiguous range of (split, row tile) pairs.
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
  Cta cta(T, a);
  const int tid = threadIdx.x;
  cta.lane = tid & 63;
  cta.w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = bx * kRT;
  // Rows past m load a valid neighbour (row m-1); they never reach Y.
  {
    const int gw = min(row0 + cta.w * Cta::RW, a.m - 1);
    cta.wavebase = a.A + (int64_t)gw * a.lda;
#pragma unroll
    for (int s = 0; s < Cta::RW; ++s)
      cta.rowoff[s] = (min(row0 + cta.w * Cta::RW + s, a.m - 1) - gw) * (int)(a.lda * 4);
  }
  const int q0 = by * a.chunks_per_split;
  const int q1 = min(q0 + a.chunks_per_split, a.total_chunks);
  // Lanes take the samples in the plan's bank-spreading order for this
  // gather (round-robin over (R_j >> 2) mod 16).
  const int lidx = (int)blockIdx.z * (NW * 64) + tid;
  cta.jok = lidx < a.l;
  cta.j = cta.jok ? a.order[lidx] : lidx;
  cta.jc = cta.jok ? cta.j : a.l - 1;
  const int rj = cta.jok ? a.R[cta.j] : 0;
  cta.pos = rj & (Cta::B - 1);
  cta.swz = (cta.pos >> 2) & 15;
  cta.rhi = (uint32_t)rj >> Cta::LOG2B;
  cta.cpb_log2 = a.log2r - Cta::LOG2B;
#pragma unroll
  for (int k = 0; k < kRT; ++k) cta.acc[k] = 0.f;

  float bufA[64], bufB[64];
  uint32_t dA[Cta::K + 1], dB[Cta::K + 1];
  // The last chunk is peeled off so that the prefetch inside the loop is
  // unconditional: with a conditional prefetch the wait inserted before the
  // sign step covers the loads just issued, which then never overlap work.
  if (q0 < q1) {
    cta.load(bufA, dA, q0);
#pragma nounroll
    for (int q = q0; q + 1 < q1; ++q) {
      cta.template step<true>(q, bufA, dA, bufB, dB);
#pragma unroll
      for (int t = 0; t < 64; ++t) bufA[t] = bufB[t];
#pragma unroll
      for (int k = 0; k <= Cta::K; ++k) dA[k] = dB[k];
    }
    cta.template step<false>(q1 - 1, bufA, dA, bufB, dB);
  }

  if (cta.jok) {
    float *o = a.out + (int64_t)by * a.split_stride + (int64_t)row0 * a.ldo + cta.j;
    const int nrow = min(kRT, a.m - row0);
#pragma unroll
    for (int k = 0; k < kRT; ++k)
      if (k < nrow) o[(int64_t)k * a.ldo] = cta.acc[k] * a.scale;
  }
}

// Direct evaluation of eq. (2.3) from the right for blocks shorter than the
// smallest chunk (2^log2r < 256; with padding, r < 2^log2r: columns
// i*r .. i*r + r - 1 of A, D signs at bits i*2^log2r + x): one thread per
// output entry, O(n) work each.
__global__ void right_direct_kernel(const float *__restrict__ A, int64_t lda, int m,
                                    const int32_t *__restrict__ R,
                                    const uint32_t *__restrict__ Dbits,
                                    const uint32_t *__restrict__ Dtbits, int64_t dt_words,
                                    int l, int64_t p, int log2r, int64_t r,
                                    float *__restrict__ Y, int64_t ldy, float scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)l * m) return;
  const int g = (int)(idx / l);
  const int j = (int)(idx - (int64_t)g * l);
  const int64_t rp = int64_t(1) << log2r;
  const uint32_t rj = (uint32_t)R[j];
  const float *row = A + (int64_t)g * lda;
  float acc = 0.f;
  for (int64_t i = 0; i < p; ++i) {
    float s = 0.f;
    for (int64_t x = 0; x < r; ++x) {
      const int64_t cd = i * rp + x;
      const uint32_t d = (Dbits[cd >> 5] >> (cd & 31)) & 1u;
      const uint32_t h = (uint32_t)__popc(rj & (uint32_t)x) & 1u;
      const float v = row[i * r + x];
      s += (d ^ h) ? -v : v;
    }
    const uint32_t dt = (Dtbits[i * dt_words + (j >> 5)] >> (j & 31)) & 1u;
    acc += dt ? -s : s;
  }
  Y[(int64_t)g * ldy + j] = acc * scale;
}

struct RightLaunch {
  bool direct = false, pad = false;
  int nw = 8;
  int rtiles = 0, groups = 0, splits = 1, cps = 0, total_chunks = 0, cr = 0;
  size_t ws = 0;
};

RightLaunch choose_right(const bsrht_plan_s *pl, int64_t m) {
  RightLaunch L;
  if (pl->rp < 256) {
    L.direct = true;
    return L;
  }
  L.pad = pl->r != pl->rp;
  L.nw = pl->rp >= 512 ? 8 : 4;
  const int b = 64 * L.nw;
  // LDS: 128 KiB per workgroup at b = 512 (one per CU), 64 KiB at b = 256.
  const int per_cu = L.nw == 8 ? 1 : 2;
  // chunks holding columns of A: all of them, or ceil(r / b) per padded block
  L.cr = (int)((pl->r + b - 1) / b);
  L.total_chunks = L.pad ? (int)(pl->p * L.cr) : (int)(pl->n / b);
  L.rtiles = (int)((m + kRT - 1) / kRT);
  const int spp = L.nw * 64;
  L.groups = (int)((pl->l + spp - 1) / spp);
  const int64_t target = (int64_t)device_cu_count() * per_cu;
  int64_t splits = target / ((int64_t)L.rtiles * L.groups);
  if (splits < 1) splits = 1;
  if (splits > L.total_chunks) splits = L.total_chunks;
  L.cps = (int)((L.total_chunks + splits - 1) / splits);
  L.splits = (L.total_chunks + L.cps - 1) / L.cps;
  L.ws = L.splits > 1 ? (size_t)L.splits * (size_t)m * (size_t)pl->l * sizeof(float) : 0;
  return L;
}

template <int NW>
int launch_right(const RightLaunch &L, const RightArgs &a, hipStream_t s) {
  dim3 grid((unsigned)L.rtiles, (unsigned)L.splits, (unsigned)L.groups);
  const int tslot = timing_begin(BSRHT_TIMING_APPLY_RIGHT, s);
  if (L.pad)
    right_fp32_kernel<NW, true><<<grid, NW * 64, 0, s>>>(a);
  else
    right_fp32_kernel<NW, false><<<grid, NW * 64, 0, s>>>(a);
  timing_end(tslot, s);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

}  // namespace

size_t apply_right_ws_bytes(const bsrht_plan_s *plan, int64_t m) {
  if (!plan || m <= 0) return 0;
  return choose_right(plan, m).ws;
}

int apply_right_fp32(const bsrht_plan_s *pl, const float *A, int64_t m, int64_t lda, float *Y,
                     int64_t ldy, void *ws, size_t ws_bytes, hipStream_t s) {
  const float scale = 1.0f / sqrtf((float)pl->l);
  const RightLaunch L = choose_right(pl, m);
  if (L.direct) {
    const int64_t total = pl->l * m;
    const int tb = 256;
    if (total > kMaxGridItems) return BSRHT_EUNSUPPORTED;
    right_direct_kernel<<<(unsigned)((total + tb - 1) / tb), tb, 0, s>>>(
        A, lda, (int)m, pl->R, pl->Dbits, pl->Dtbits, pl->dt_words, (int)pl->l, pl->p,
        pl->log2r, pl->r, Y, ldy, scale);
    BSRHT_LAUNCH_CHECK();
    return BSRHT_OK;
  }
  if (L.groups > 65535 || L.rtiles > INT_MAX / kRT) return BSRHT_EUNSUPPORTED;
  // One wave's rows are addressed by 32-bit byte offsets from its first row.
  if ((int64_t)(kRT / L.nw) * lda * 4 >= (int64_t(1) << 31)) return BSRHT_EUNSUPPORTED;
  if (ws_bytes < L.ws || (L.ws && !ws)) return BSRHT_ENOMEM;
  RightArgs a;
  a.A = A;
  a.lda = lda;
  a.m = (int)m;
  a.R = pl->R;
  a.order = pl->order_right;
  a.Dbits = pl->Dbits;
  a.Dtbits = pl->Dtbits;
  a.dt_words = (int)pl->dt_words;
  a.l = (int)pl->l;
  a.log2r = pl->log2r;
  a.chunks_per_split = L.cps;
  a.total_chunks = L.total_chunks;
  a.r_cols = pl->r;
  a.cr = L.cr;
  if (L.splits > 1) {
    a.out = static_cast<float *>(ws);
    a.ldo = pl->l;
    a.split_stride = m * pl->l;
    a.scale = 1.0f;
  } else {
    a.out = Y;
    a.ldo = ldy;
    a.split_stride = 0;
    a.scale = scale;
  }
  BSRHT_TRY(L.nw == 8 ? launch_right<8>(L, a, s) : launch_right<4>(L, a, s));
  if (L.splits > 1)
    return reduce_splits(static_cast<const float *>(ws), L.splits, m * pl->l, m, pl->l, Y, ldy,
                         scale, s);
  return BSRHT_OK;
}

}  // namespace bsrht

using namespace bsrht;

extern "C" {

size_t bsrht_apply_right_workspace(bsrht_plan_t plan, int64_t m) {
  return apply_right_ws_bytes(plan, m);
}

int bsrht_apply_right(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda, float *Y,
                      int64_t ldy, void *ws, size_t ws_bytes, void *stream) {
  if (!plan || m < 0) return BSRHT_EINVAL;
  if (m == 0) return BSRHT_OK;
  if (!A || !Y || lda < plan->n || ldy < plan->l || m > INT_MAX) return BSRHT_EINVAL;
  if ((int64_t)plan->l * m > ((int64_t)1 << 40)) return BSRHT_EUNSUPPORTED;
  return apply_right_fp32(plan, A, m, lda, Y, ldy, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
