// Fused block SRHT apply, FP32 butterflies: Y = Omega A (section 2,
// eq. (2.3)-(2.4)) for row-major A (n x m).
//
// Structure.  H_r factors as H_{r/b} (x) H_b for the index split
// x = x_hi*b + x_lo (Kronecker form of H, section 2).  A workgroup of NW waves
// (8, or 16 when l > 512 so that one thread serves each sample) owns 64
// columns (lane = column) and streams chunks of b = NW*BR consecutive rows
// (one chunk = one x_hi of one block i); wave w holds chunk rows
// x_lo = w*BR + t, t in [0, BR), in registers.  For each chunk:
//   1. load  : non-temporal buffer loads, one 256-byte row segment per
//              wave instruction; the next chunk is already in flight;
//   2. D^(i) : sign flips, wave-uniform per row (sign-bit xor);
//   3. H_BR  : log2(BR) radix-2 stages over t, in registers;
//   4. H_NW  : one LDS exchange, log2(NW) stages over w (rows t + BR*k);
//              the chunk now holds H_b applied to each column;
//   5. gather: lane = sample j; only the l sampled outputs are needed,
//              (H_r v)[R_j] = sum_{x_hi} (-1)^popcount(R_j,hi & x_hi)
//                             * (H_b v_{x_hi})[R_j,lo],
//              so each sample adds +-row R_j,lo of the chunk (float4 LDS
//              reads) with sign Dt^(i)_j * (-1)^popcount(R_j,hi & x_hi).
// The accumulators run across chunks and across blocks, so the sum over
// blocks (2.4) happens in registers; no transformed block is ever written to
// HBM.  A is read exactly once.  Row splits (for parallelism) write l x m
// partials that a second kernel sums in fixed split order and scales by
// 1/sqrt(l) (the product sqrt(r/l) * 1/sqrt(r) of eq. (2.3)).
// The 16-wave instances (256-row chunks, 68 KiB of LDS) write the exchange's
// output to a second LDS buffer that the gather reads, so the next chunk's
// stores cannot race the gather and one of the three barriers per chunk
// goes; the 8-wave chunk (139 KiB) leaves no room for a second buffer.
#include <limits.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace bsrht {
namespace {

constexpr int kCT = 64;         // columns per workgroup (one per lane)
constexpr int kLDT = kCT + 4;   // LDS row stride in floats (272 B, float4 aligned)
constexpr int kBufDword3 = 0x00020000;  // raw buffer resource word 3 (gfx9 family)
constexpr int kAuxNT = 2;       // buffer cache policy: non-temporal (A is read once)

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

struct FusedArgs {
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
  int64_t r_rows;  // rows per block in A (padded plans: r < 2^log2r)
  int cr;          // chunks per block that hold rows of A (padded plans)
  const int32_t *order;  // sample of each gather lane
};

// Unscaled Walsh-Hadamard transform of N values held in registers.
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

// Rows T0 .. T1-1 of the BR consecutive rows starting at `base`
// (wave-uniform); voff = column bytes.
template <int BR, int T0 = 0, int T1 = BR>
__device__ __forceinline__ void load_rows(float (&v)[BR], const float *base, int voff,
                                          int row_bytes) {
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(base);
#pragma unroll
  for (int t = T0; t < T1; ++t)
    v[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, t * row_bytes, kAuxNT));
}

// The same for a wave whose first vr rows (wave-uniform, 0 <= vr <= BR) hold
// data and the rest are the zero padding of a block: row t >= vr is read at
// row max(vr - 1, 0), an address inside A.  The caller zeroes those rows when
// it uses them (doing it here would make the wave wait for the loads).
template <int BR, int T0 = 0, int T1 = BR>
__device__ __forceinline__ void load_rows_clamped(float (&v)[BR], const float *base, int voff,
                                                  int row_bytes, int vr) {
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(base);
  const int last = vr > 0 ? vr - 1 : 0;
#pragma unroll
  for (int t = T0; t < T1; ++t) {
    const int tr = t < last ? t : last;
    v[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, tr * row_bytes, kAuxNT));
  }
}

// D^(i) for global rows g0 .. g0+BR-1 (g0 a multiple of BR, wave-uniform):
// flip the sign bit where the table bit is set.
template <int BR>
__device__ __forceinline__ void apply_dsigns(float (&v)[BR], const uint32_t *__restrict__ Dbits,
                                             int64_t g0) {
  if constexpr (BR >= 32) {
#pragma unroll
    for (int wd = 0; wd < BR / 32; ++wd) {
      const uint32_t bits = Dbits[(g0 >> 5) + wd];
#pragma unroll
      for (int b = 0; b < 32; ++b) {
        const uint32_t msk = (bits << (31 - b)) & 0x80000000u;
        v[wd * 32 + b] = __uint_as_float(__float_as_uint(v[wd * 32 + b]) ^ msk);
      }
    }
  } else {
    const uint32_t bits = Dbits[g0 >> 5] >> (uint32_t)(g0 & 31);
#pragma unroll
    for (int b = 0; b < BR; ++b) {
      const uint32_t msk = (bits << (31 - b)) & 0x80000000u;
      v[b] = __uint_as_float(__float_as_uint(v[b]) ^ msk);
    }
  }
}

// PAD: a plan whose blocks hold r rows of A, padded with zeros to
// rp = 2^log2r.  The split ranges count the chunks that hold rows of A
// (cr per block); chunk qr of them is chunk qp = i*(rp/B) + xhi of the padded
// layout (signs, block index and H_{r/b} sign use qp), stored at row
// i*r + xhi*B of A, with the rows past r read as zeros.
template <int NW, int BR, bool PAD = false>
struct FusedCta {
  static constexpr int B = BR * NW;
  static constexpr int LOG2B = ilog2c(B);
  static constexpr int G = BR / NW;  // radix-NW groups per wave
  static_assert(G >= 1, "need BR >= NW");

  float *T;
  float *T2 = nullptr;  // second buffer: exchange output, gather input
  const FusedArgs &a;
  int lane, w, j, pos, cpb_log2, voff, row_bytes;
  bool jok;
  uint32_t rhi;  // R_j's chunk-index bits (R_j >> log2 b)
  int cur_block;
  uint32_t dtbit;
  const float *wavebase;  // A + c0 + w*BR*lda (wave-uniform)
  const float *tilebase;  // A + c0
  float acc[kCT];

  __device__ __forceinline__ FusedCta(float *T_, const FusedArgs &a_) : T(T_), a(a_) {}

  __device__ __forceinline__ const float *chunk_base(int q) const {
    return wavebase + (int64_t)q * B * a.lda;
  }

  // PAD: the current chunk is chunk cx of block ci (chunk ci*(rp/B) + cx of
  // the padded layout; its rows start at row ci*r + cx*B of A), and cvr of
  // this wave's rows hold data.  (ci, cx) advance by one chunk per step, so
  // no division runs per chunk; the next chunk's address is ready before its
  // loads are issued.
  int ci = 0, cx = 0, cvr = BR;
  // Where this wave's rows of chunk x of block i start in A and how many
  // hold data (with none, the tile's first row of A, which always exists,
  // stands in as the address).  Every quantity is wave-uniform;
  // readfirstlane states it, so the row offsets stay scalar.
  __device__ __forceinline__ const float *padded_base(int i, int x, int &vr) const {
    int64_t v = a.r_rows - (int64_t)x * B - w * BR;
    v = v < 0 ? 0 : (v > BR ? BR : v);
    vr = __builtin_amdgcn_readfirstlane((int)v);
    if (vr == 0) return tilebase;
    const int64_t row = (int64_t)i * a.r_rows + (int64_t)x * B;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)row);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)row >> 32));
    return wavebase + (int64_t)(((uint64_t)hi << 32) | lo) * a.lda;
  }
  // First chunk q0 of this workgroup's range.
  __device__ __forceinline__ void load_first(float (&v)[BR], int q0) {
    if constexpr (PAD) {
      ci = __builtin_amdgcn_readfirstlane(q0 / a.cr);
      cx = q0 - ci * a.cr;
      const float *base = padded_base(ci, cx, cvr);
      load_rows_clamped<BR>(v, base, voff, row_bytes, cvr);
    } else {
      load_rows<BR>(v, chunk_base(q0), voff, row_bytes);
    }
  }

  __device__ __forceinline__ void step(int qr, int q1, float (&cur)[BR], float (&nxt)[BR]) {
    // The next chunk is prefetched in two halves: the second half is issued
    // once this chunk's rows have left the registers for LDS, which keeps
    // the accumulators, one chunk and half a chunk within 256 VGPRs.
    const bool more = qr + 1 < q1;
    int q = qr;
    int ni = 0, nx = 0, nvr = BR;
    const float *nbase = nullptr;
    if constexpr (PAD) {
      q = (ci << cpb_log2) + cx;
      ni = cx + 1 == a.cr ? ci + 1 : ci;
      nx = cx + 1 == a.cr ? 0 : cx + 1;
      if (more) nbase = padded_base(ni, nx, nvr);
      if (more) load_rows_clamped<BR, 0, BR / 2>(nxt, nbase, voff, row_bytes, nvr);
#pragma unroll
      for (int t = 0; t < BR; ++t)  // the block's zero padding
        if (t >= cvr) cur[t] = 0.f;
    } else {
      if (more) load_rows<BR, 0, BR / 2>(nxt, chunk_base(qr + 1), voff, row_bytes);
    }
    apply_dsigns<BR>(cur, a.Dbits, (int64_t)q * B + w * BR);
    fwht_regs<BR>(cur);
    {
      float *Tw = T + (w * BR) * kLDT + lane;
#pragma unroll
      for (int t = 0; t < BR; ++t) Tw[t * kLDT] = cur[t];
    }
    if constexpr (PAD) {
      if (more) load_rows_clamped<BR, BR / 2, BR>(nxt, nbase, voff, row_bytes, nvr);
      ci = ni;
      cx = nx;
      cvr = nvr;
    } else {
      if (more) load_rows<BR, BR / 2, BR>(nxt, chunk_base(qr + 1), voff, row_bytes);
    }
    __syncthreads();
    // H_NW over w: group t holds rows t, t+BR, ..., t+(NW-1)*BR.
    float *const Tx = T2 ? T2 : T;  // where the exchange writes and the gather reads
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const float *Tg = T + (w * G + g) * kLDT + lane;
      float *Og = Tx + (w * G + g) * kLDT + lane;
      float v[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) v[k] = Tg[k * BR * kLDT];
      fwht_regs<NW>(v);
#pragma unroll
      for (int k = 0; k < NW; ++k) Og[k * BR * kLDT] = v[k];
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
        const float4 v = row[c4];
        acc[4 * c4 + 0] = fmaf(sgn, v.x, acc[4 * c4 + 0]);
        acc[4 * c4 + 1] = fmaf(sgn, v.y, acc[4 * c4 + 1]);
        acc[4 * c4 + 2] = fmaf(sgn, v.z, acc[4 * c4 + 2]);
        acc[4 * c4 + 3] = fmaf(sgn, v.w, acc[4 * c4 + 3]);
      }
    }
    // With one buffer the next chunk's stores must wait for every gather.
    // With two, the next exchange writes T2 only after the next chunk's
    // first barrier, which every wave passes after this gather.
    if (!T2) __syncthreads();
  }
};

// One workgroup's share of a launch: column tile bx, row split by, sample
// group bz (T: the chunk buffer in LDS, NW*BR*kLDT floats).  Shared by the
// single-job kernel and the persistent batch kernel, so that a job's result
// does not depend on which of them ran it.
template <int NW, int BR, bool PAD = false>
__device__ __forceinline__ void fused_tile(const FusedArgs &a, float *T, int bx, int by, int bz,
                                           float *T2 = nullptr) {
  using Cta = FusedCta<NW, BR, PAD>;
  Cta cta(T, a);
  cta.T2 = T2;
  const int tid = threadIdx.x;
  cta.lane = tid & 63;
  cta.w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c0 = bx * kCT;
  // Columns past m load a valid neighbour (column m-1); they never reach Y.
  const int cc = min(c0 + cta.lane, a.m - 1) - c0;
  cta.voff = cc * 4;
  cta.row_bytes = (int)(a.lda * 4);
  cta.wavebase = a.A + c0 + (int64_t)(cta.w * BR) * a.lda;
  cta.tilebase = a.A + c0;
  const int q0 = by * a.chunks_per_split;
  const int q1 = min(q0 + a.chunks_per_split, a.total_chunks);
  // Lanes take the samples in the plan's bank-spreading order (round-robin
  // over R_j mod 16, the gather's LDS bank group).
  const int lidx = bz * (NW * 64) + tid;
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

  // One step per iteration and an explicit copy of the prefetched chunk: with
  // two alternating step bodies the register allocator ran out of the 256
  // registers and spilled R_j's chunk bits, whose reload in the gather (a
  // vector-memory access) waited for the whole prefetch of the next chunk.
  float bufA[BR], bufB[BR];
  if (q0 < q1) cta.load_first(bufA, q0);
#pragma nounroll
  for (int q = q0; q < q1; ++q) {
    cta.step(q, q1, bufA, bufB);
#pragma unroll
    for (int t = 0; t < BR; ++t) bufA[t] = bufB[t];
  }

  if (cta.jok) {
    float *o = a.out + (int64_t)by * a.split_stride + (int64_t)cta.j * a.ldo + c0;
    const int ncol = min(kCT, a.m - c0);
#pragma unroll
    for (int k = 0; k < kCT; ++k)
      if (k < ncol) o[k] = cta.acc[k] * a.scale;
  }
}

template <int NW, int BR, bool PAD = false>
__global__ __launch_bounds__(NW * 64) void fused_fp32_kernel(FusedArgs a) {
  constexpr bool DB = NW == 16;  // two LDS buffers (see the file comment)
  __shared__ __attribute__((aligned(16))) float T[(DB ? 2 : 1) * NW * BR * kLDT];
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs round-robin, so
  // linear id k runs on XCD k mod 8; give each XCD a contiguous range of
  // (split, column tile) pairs in row-major order.
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
  fused_tile<NW, BR, PAD>(a, T, bx, by, (int)blockIdx.z, DB ? T + NW * BR * kLDT : nullptr);
}

// Y[j, c] = scale * sum_s part[s][j][c], splits summed in ascending order.
__global__ void reduce_splits_kernel(const float *__restrict__ part, int splits,
                                     int64_t split_stride, int l, int m,
                                     float *__restrict__ Y, int64_t ldy, float scale) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)l * m;
       idx += stride) {
    const int j = (int)(idx / m);
    const int c = (int)(idx - (int64_t)j * m);
    const float *p = part + (int64_t)j * m + c;
    float s = 0.f;
    for (int sp = 0; sp < splits; ++sp) s += p[(int64_t)sp * split_stride];
    Y[(int64_t)j * ldy + c] = s * scale;
  }
}

// Direct evaluation of eq. (2.3) for blocks shorter than the smallest fused
// chunk (2^log2r < 64): one thread per output entry, O(n) work each.  Block i
// holds rows i*r .. i*r + r - 1 of A (r < 2^log2r: zero padding, whose rows
// contribute nothing); its D signs sit at bits i*2^log2r + x.
__global__ void direct_kernel(const float *__restrict__ A, int64_t lda, int m,
                              const int32_t *__restrict__ R, const uint32_t *__restrict__ Dbits,
                              const uint32_t *__restrict__ Dtbits, int64_t dt_words, int l,
                              int64_t p, int log2r, int64_t r, float *__restrict__ Y, int64_t ldy,
                              float scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)l * m) return;
  const int j = (int)(idx / m);
  const int c = (int)(idx - (int64_t)j * m);
  const int64_t rp = int64_t(1) << log2r;
  const uint32_t rj = (uint32_t)R[j];
  float acc = 0.f;
  for (int64_t i = 0; i < p; ++i) {
    float s = 0.f;
    for (int64_t x = 0; x < r; ++x) {
      const int64_t gd = i * rp + x;
      const uint32_t d = (Dbits[gd >> 5] >> (gd & 31)) & 1u;
      const uint32_t h = (uint32_t)__popc(rj & (uint32_t)x) & 1u;
      const float v = A[(i * r + x) * lda + c];
      s += (d ^ h) ? -v : v;
    }
    const uint32_t dt = (Dtbits[i * dt_words + (j >> 5)] >> (j & 31)) & 1u;
    acc += dt ? -s : s;
  }
  Y[(int64_t)j * ldy + c] = acc * scale;
}

struct Launch {
  bool direct = false;
  int nw = 8, br = 0, b = 0;
  int ctiles = 0, groups = 0, splits = 1, cps = 0, total_chunks = 0;
  size_t ws = 0;
};

Launch choose_launch(const bsrht_plan_s *pl, int64_t m, int64_t lda) {
  Launch L;
  (void)lda;
  int per_cu;
  if (pl->l > 512 && pl->rp >= 256) {
    // 16 waves, one thread per sample for l <= 1024: A is read once per
    // 1024 samples instead of once per 512; chunks of b = 16*16 rows.
    L.nw = 16;
    L.br = 16;
    per_cu = 1;  // 1024 threads at ~100 VGPRs fill the register file
  } else {
    // Largest chunk b = 8*BR <= r with 8 <= BR <= 64.
    int br = 64;
    while (br >= 8 && (int64_t)br * 8 > pl->rp) br >>= 1;
    if (br < 8) {
      L.direct = true;
      return L;
    }
    L.nw = 8;
    L.br = br;
    per_cu = br * 8 * kLDT * 4 > 80 * 1024 ? 1 : 2;
  }
  L.b = L.br * L.nw;
  // Chunks that hold rows of A: all of them, or ceil(r / b) per padded block.
  L.total_chunks = (int)(pl->p * ((pl->r + L.b - 1) / L.b));
  L.ctiles = (int)((m + kCT - 1) / kCT);
  const int spp = L.nw * 64;
  L.groups = (int)((pl->l + spp - 1) / spp);
  const int64_t target = (int64_t)device_cu_count() * per_cu;
  int64_t splits = target / ((int64_t)L.ctiles * L.groups);
  if (splits < 1) splits = 1;
  if (splits > L.total_chunks) splits = L.total_chunks;
  L.cps = (int)((L.total_chunks + splits - 1) / splits);
  L.splits = (L.total_chunks + L.cps - 1) / L.cps;
  L.ws = L.splits > 1 ? (size_t)L.splits * (size_t)pl->l * (size_t)m * sizeof(float) : 0;
  return L;
}

template <int NW, int BR, bool PAD = false>
int launch_fused(const Launch &L, FusedArgs &a, hipStream_t s) {
  dim3 grid((unsigned)L.ctiles, (unsigned)L.splits, (unsigned)L.groups);
  const int tslot = timing_begin(BSRHT_TIMING_APPLY_FP32, s);
  fused_fp32_kernel<NW, BR, PAD><<<grid, NW * 64, 0, s>>>(a);
  timing_end(tslot, s);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

// ---------------------------------------------------------------------------
// Batches of small sketches: one persistent launch per workgroup shape runs
// the workgroup tiles of every job in the batch, read from a descriptor table
// in device memory, and one persistent launch sums the row-split partials.
// Each job keeps exactly the launch decomposition bsrht_apply would use (the
// same template instance, chunk ranges, row splits and summation order), so
// its result is bitwise the single call's.
constexpr int kBatchMax = BSRHT_BATCH_MAX;

struct BatchItem {
  FusedArgs a;          // the single-job launch's arguments
  int br, ctiles, splits, groups;
  int wg_begin;         // first work item of the job in its list
  int64_t red_begin;    // first element of the job in the reduce (splits > 1)
  const float *part;    // row-split partials (splits > 1)
  float *Y;
  int64_t ldy;
  int l, m;
  int64_t split_stride;
  float scale;
};

struct BatchList {  // jobs of one workgroup shape (8 or 16 waves)
  int count, total_wg;
  int64_t total_red;
  BatchItem items[kBatchMax];
};

struct BatchTable {
  BatchList nw8, nw16;
};

template <int NW>
__global__ __launch_bounds__(NW * 64) void fused_batch_kernel(const BatchList *__restrict__ L) {
  __shared__ __attribute__((aligned(16))) float T[(NW == 8 ? 8 * 64 : 16 * 16) * kLDT];
  const int total = L->total_wg, count = L->count;
  for (int w = (int)blockIdx.x; w < total; w += (int)gridDim.x) {
    int k = 0;  // the job whose work items contain w
    while (k + 1 < count && L->items[k + 1].wg_begin <= w) ++k;
    const BatchItem &it = L->items[k];
    int loc = w - it.wg_begin;
    const int bx = loc % it.ctiles;
    loc /= it.ctiles;
    const int by = loc % it.splits, bz = loc / it.splits;
    const FusedArgs a = it.a;
    if constexpr (NW == 16) {
      fused_tile<16, 16>(a, T, bx, by, bz);
    } else {
      switch (it.br) {
        case 64: fused_tile<8, 64>(a, T, bx, by, bz); break;
        case 32: fused_tile<8, 32>(a, T, bx, by, bz); break;
        case 16: fused_tile<8, 16>(a, T, bx, by, bz); break;
        default: fused_tile<8, 8>(a, T, bx, by, bz); break;
      }
    }
    __syncthreads();  // the next work item reuses T
  }
}

// Y = scale * (sum of the splits in ascending order), as reduce_splits_kernel,
// over the partials of every job of both lists.
__global__ void reduce_batch_kernel(const BatchTable *__restrict__ tb) {
  const int64_t n8 = tb->nw8.total_red, total = n8 + tb->nw16.total_red;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const BatchList &L = idx < n8 ? tb->nw8 : tb->nw16;
    const int64_t e = idx < n8 ? idx : idx - n8;
    int k = 0;  // the last job whose elements start at or before e
    while (k + 1 < L.count && L.items[k + 1].red_begin <= e) ++k;
    const BatchItem &it = L.items[k];
    const int64_t loc = e - it.red_begin;
    const int j = (int)(loc / it.m);
    const int c = (int)(loc - (int64_t)j * it.m);
    const float *pp = it.part + (int64_t)j * it.m + c;
    float sum = 0.f;
    for (int sp = 0; sp < it.splits; ++sp) sum += pp[(int64_t)sp * it.split_stride];
    it.Y[(int64_t)j * it.ldy + c] = sum * it.scale;
  }
}

}  // namespace

size_t apply_fp32_ws_bytes(const bsrht_plan_s *plan, int64_t m) {
  if (!plan || m <= 0) return 0;
  return choose_launch(plan, m, m).ws;
}

size_t apply_ws_bytes(const bsrht_plan_s *plan, int64_t m) {
  if (!plan || m <= 0) return 0;
  if (plan->precision == BSRHT_SPLIT_BF16) return apply_split_bf16_ws_bytes(plan, m);
  return apply_fp32_ws_bytes(plan, m);
}

int reduce_splits(const float *part, int splits, int64_t split_stride, int64_t l, int64_t m,
                  float *Y, int64_t ldy, float scale, hipStream_t s) {
  const int64_t total = l * m;
  const int tb = 256;
  reduce_splits_kernel<<<stride_grid(total, tb), tb, 0, s>>>(
      part, splits, split_stride, (int)l, (int)m, Y, ldy, scale);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

namespace {

// The fused launch's arguments for one sketch (checks the launch limits and
// the workspace).
int fused_args(const bsrht_plan_s *pl, const float *A, int64_t m, int64_t lda, float *Y,
               int64_t ldy, void *ws, size_t ws_bytes, const Launch &L, FusedArgs &a) {
  if (L.groups > 65535 || L.ctiles <= 0) return BSRHT_EUNSUPPORTED;
  // Row offsets inside one wave's BR rows are 32-bit buffer offsets.
  if ((int64_t)L.br * lda * 4 >= (int64_t(1) << 31)) return BSRHT_EUNSUPPORTED;
  if (ws_bytes < L.ws || (L.ws && !ws)) return BSRHT_ENOMEM;
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
  a.r_rows = pl->r;
  a.cr = (int)((pl->r + L.b - 1) / L.b);
  if (L.splits > 1) {
    a.out = static_cast<float *>(ws);
    a.ldo = m;
    a.split_stride = pl->l * m;
    a.scale = 1.0f;
  } else {
    a.out = Y;
    a.ldo = ldy;
    a.split_stride = 0;
    a.scale = 1.0f / sqrtf((float)pl->l);
  }
  return BSRHT_OK;
}

// The batch's two persistent sketch launches and its reduce, captured once
// per (device, descriptor table) into a graph that later calls replay: the
// kernels read everything else from the table.
// Each entry also owns the pinned staging of the table's descriptors and an
// event recorded after their copy, so the staging is rewritten only once
// the previous copy has run.
struct BatchGraph {
  int device;
  const void *table;
  hipGraphExec_t exec;
  char *pinned;
  hipEvent_t copied;
};
std::mutex g_batch_mu;
std::vector<BatchGraph> g_batch_graphs;

int batch_graph(const void *table, BatchGraph *out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BSRHT_EDEVICE;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (const BatchGraph &g : g_batch_graphs)
    if (g.device == dev && g.table == table) {
      *out = g;
      return BSRHT_OK;
    }
  void *pin = nullptr;
  hipEvent_t ev = nullptr;
  if (hipHostMalloc(&pin, sizeof(BatchTable), hipHostMallocDefault) != hipSuccess)
    return BSRHT_EDEVICE;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(pin);
    return BSRHT_EDEVICE;
  }
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    (void)hipEventDestroy(ev);
    (void)hipHostFree(pin);
    return BSRHT_EDEVICE;
  }
  const BatchTable *tb = static_cast<const BatchTable *>(table);
  const unsigned cus = (unsigned)device_cu_count();
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    fused_batch_kernel<8><<<cus, 8 * 64, 0, cs>>>(&tb->nw8);
    fused_batch_kernel<16><<<cus, 16 * 64, 0, cs>>>(&tb->nw16);
    reduce_batch_kernel<<<4 * cus, 256, 0, cs>>>(tb);
    ok = hipGetLastError() == hipSuccess;
    ok = hipStreamEndCapture(cs, &graph) == hipSuccess && ok;
  }
  ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  if (!ok) {
    (void)hipEventDestroy(ev);
    (void)hipHostFree(pin);
    return BSRHT_EDEVICE;
  }
  g_batch_graphs.push_back({dev, table, exec, static_cast<char *>(pin), ev});
  *out = g_batch_graphs.back();
  return BSRHT_OK;
}

}  // namespace

// Destroys the graph, event and pinned staging of one table on the current
// device (all = false) or of every table on every device (all = true).  The
// caller guarantees that no launch through these tables is still pending;
// the copy event is waited for regardless.
int release_batch_graphs(const void *table, bool all) {
  int dev = 0;
  if (!all && hipGetDevice(&dev) != hipSuccess) return BSRHT_EDEVICE;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  int st = BSRHT_OK;
  for (size_t i = 0; i < g_batch_graphs.size();) {
    const BatchGraph &g = g_batch_graphs[i];
    if (!all && (g.device != dev || g.table != table)) {
      ++i;
      continue;
    }
    if (hipEventSynchronize(g.copied) != hipSuccess) st = BSRHT_EDEVICE;
    if (hipGraphExecDestroy(g.exec) != hipSuccess) st = BSRHT_EDEVICE;
    if (hipEventDestroy(g.copied) != hipSuccess) st = BSRHT_EDEVICE;
    if (hipHostFree(g.pinned) != hipSuccess) st = BSRHT_EDEVICE;
    g_batch_graphs.erase(g_batch_graphs.begin() + (std::ptrdiff_t)i);
  }
  return st;
}

int apply_fp32(const bsrht_plan_s *pl, const float *A, int64_t m, int64_t lda, float *Y,
               int64_t ldy, void *ws, size_t ws_bytes, hipStream_t s) {
  const float scale = 1.0f / sqrtf((float)pl->l);
  const Launch L = choose_launch(pl, m, lda);
  if (L.direct) {
    const int64_t total = pl->l * m;
    const int tb = 256;
    if (total > kMaxGridItems) return BSRHT_EUNSUPPORTED;
    direct_kernel<<<(unsigned)((total + tb - 1) / tb), tb, 0, s>>>(
        A, lda, (int)m, pl->R, pl->Dbits, pl->Dtbits, pl->dt_words, (int)pl->l, pl->p,
        pl->log2r, pl->r, Y, ldy, scale);
    BSRHT_LAUNCH_CHECK();
    return BSRHT_OK;
  }
  FusedArgs a;
  {
    const int st = fused_args(pl, A, m, lda, Y, ldy, ws, ws_bytes, L, a);
    if (st != BSRHT_OK) return st;
  }
  int st;
  if (pl->r != pl->rp) {  // padded blocks: their own instances
    if (L.nw == 16) {
      st = launch_fused<16, 16, true>(L, a, s);
    } else {
      switch (L.br) {
        case 64: st = launch_fused<8, 64, true>(L, a, s); break;
        case 32: st = launch_fused<8, 32, true>(L, a, s); break;
        case 16: st = launch_fused<8, 16, true>(L, a, s); break;
        default: st = launch_fused<8, 8, true>(L, a, s); break;
      }
    }
  } else if (L.nw == 16) {
    st = launch_fused<16, 16>(L, a, s);
  } else {
    switch (L.br) {
      case 64: st = launch_fused<8, 64>(L, a, s); break;
      case 32: st = launch_fused<8, 32>(L, a, s); break;
      case 16: st = launch_fused<8, 16>(L, a, s); break;
      default: st = launch_fused<8, 8>(L, a, s); break;
    }
  }
  if (st != BSRHT_OK) return st;
  if (L.splits > 1)
    return reduce_splits(static_cast<const float *>(ws), L.splits, pl->l * m, pl->l, m, Y, ldy,
                         scale, s);
  return BSRHT_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free sketch: the row-split partials of bsrht_apply live in a
// file-scope device array instead of a caller's workspace.  Host code never
// passes the array's name to a kernel (on the host that name is a stand-in,
// not a device address): the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and is kept per device.
constexpr size_t kNoAllocScratchBytes = BSRHT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`.
int scratch_address(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BSRHT_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return BSRHT_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BSRHT_OK;
}
}  // namespace

}  // namespace bsrht

using namespace bsrht;

extern "C" {

size_t bsrht_apply_workspace(bsrht_plan_t plan, int64_t m) { return apply_ws_bytes(plan, m); }

int bsrht_apply_noalloc(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda, float *Y,
                        int64_t ldy, void *stream) {
  if (!plan || m < 0) return BSRHT_EINVAL;
  if (m == 0) return BSRHT_OK;
  if (!A || !Y || lda < m || ldy < m || m > INT_MAX) return BSRHT_EINVAL;
  if ((int64_t)plan->l * m > ((int64_t)1 << 40)) return BSRHT_EUNSUPPORTED;
  const size_t need = apply_ws_bytes(plan, m);
  if (need > kNoAllocScratchBytes) return BSRHT_ENOMEM;
  void *ws = nullptr;
  if (need > 0) {
    const int st = scratch_address(&ws);
    if (st != BSRHT_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  if (plan->precision == BSRHT_SPLIT_BF16)
    return apply_split_bf16(plan, A, m, lda, Y, ldy, ws, need, s);
  return apply_fp32(plan, A, m, lda, Y, ldy, ws, need, s);
}

int bsrht_apply(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda, float *Y,
                int64_t ldy, void *ws, size_t ws_bytes, void *stream) {
  if (!plan || m < 0) return BSRHT_EINVAL;
  if (m == 0) return BSRHT_OK;
  if (!A || !Y || lda < m || ldy < m || m > INT_MAX) return BSRHT_EINVAL;
  if ((int64_t)plan->l * m > ((int64_t)1 << 40)) return BSRHT_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  if (plan->precision == BSRHT_SPLIT_BF16)
    return apply_split_bf16(plan, A, m, lda, Y, ldy, ws, ws_bytes, s);
  return apply_fp32(plan, A, m, lda, Y, ldy, ws, ws_bytes, s);
}

size_t bsrht_batch_table_bytes(void) { return sizeof(BatchTable); }

int bsrht_batch_table_release(void *table) {
  if (!table) return BSRHT_EINVAL;
  return release_batch_graphs(table, false);
}

int bsrht_apply_batch(const bsrht_apply_item_t *items, int count, void *table,
                      size_t table_bytes, void *stream) {
  if (count < 0 || count > kBatchMax || (count > 0 && !items) || !table ||
      table_bytes < sizeof(BatchTable))
    return BSRHT_EINVAL;
  if (count == 0) return BSRHT_OK;
  std::vector<char> hbuf(sizeof(BatchTable), 0);
  BatchTable &h = *reinterpret_cast<BatchTable *>(hbuf.data());
  for (int i = 0; i < count; ++i) {
    const bsrht_apply_item_t &in = items[i];
    const bsrht_plan_s *pl = in.plan;
    const int64_t m = in.m;
    if (!pl || m < 1 || !in.A || !in.Y || in.lda < m || in.ldy < m || m > INT_MAX)
      return BSRHT_EINVAL;
    if (pl->precision != BSRHT_FP32 || pl->r != pl->rp || pl->l * m > ((int64_t)1 << 40))
      return BSRHT_EUNSUPPORTED;
    const Launch L = choose_launch(pl, m, in.lda);
    if (L.direct) return BSRHT_EUNSUPPORTED;
    BatchList &bl = L.nw == 16 ? h.nw16 : h.nw8;
    BatchItem &it = bl.items[bl.count];
    const int st = fused_args(pl, in.A, m, in.lda, in.Y, in.ldy, in.ws, in.ws_bytes, L, it.a);
    if (st != BSRHT_OK) return st;
    const int64_t wgs = (int64_t)L.ctiles * L.splits * L.groups;
    if (bl.total_wg + wgs > INT_MAX) return BSRHT_EUNSUPPORTED;
    it.br = L.br;
    it.ctiles = L.ctiles;
    it.splits = L.splits;
    it.groups = L.groups;
    it.wg_begin = bl.total_wg;
    bl.total_wg += (int)wgs;
    it.red_begin = bl.total_red;
    it.part = static_cast<const float *>(in.ws);
    it.Y = in.Y;
    it.ldy = in.ldy;
    it.l = (int)pl->l;
    it.m = (int)m;
    it.split_stride = pl->l * m;
    it.scale = 1.0f / sqrtf((float)pl->l);
    if (L.splits > 1) bl.total_red += pl->l * m;
    ++bl.count;
  }
  hipStream_t s = (hipStream_t)stream;
  BatchGraph g;
  BSRHT_TRY(batch_graph(table, &g));
  if (hipEventSynchronize(g.copied) != hipSuccess) return BSRHT_EDEVICE;
  std::memcpy(g.pinned, hbuf.data(), sizeof(BatchTable));
  if (hipMemcpyAsync(table, g.pinned, sizeof(BatchTable), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipEventRecord(g.copied, s) != hipSuccess || hipGraphLaunch(g.exec, s) != hipSuccess)
    return BSRHT_EDEVICE;
  return BSRHT_OK;
}

}  // extern "C"
