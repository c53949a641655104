// pack.hip -- per-run initialisation, class partition and bit packing.
//
// Genotype tables (section 3.1, Fig. 2): one binary row per genotype value and
// variant, columns = samples segregated into controls then cases, 64 samples
// per 64-bit word (section 4, data/bit-level parallelism).  Bit b of word w of
// class c is the sample at class position 64 w + b.  Padding bits are zero in
// every row, so the third row is stored as valid & ~(row0 | row1).
#include "device_common.hpp"

namespace fiuncho {

// Clears every job's run state, survivor histograms, class counts and pilot
// score slots, and the tile counters: workgroups (job, y) share the large
// clears, y = 0 does the rest.
// (A fill kernel rather than hipMemsetAsync, so that the sequence can be
// captured into a graph and replayed.)
constexpr int kInitBlocks = 32;
__global__ void init_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.x];
  const uint32_t t = blockIdx.y * blockDim.x + threadIdx.x, nt = gridDim.y * blockDim.x;
  for (uint32_t i = t; i < J.n * 6; i += nt) J.marg[i] = 0;
  {
    uint4 *pk = reinterpret_cast<uint4 *>(J.cand);
    const uint32_t n4 = J.pilot_slots / 4;
    for (uint32_t i = t; i < n4; i += nt) pk[i] = make_uint4(0, 0, 0, 0);
  }
  if (blockIdx.y != 0) return;
  for (uint32_t i = threadIdx.x; i < (uint32_t)kHistBins; i += blockDim.x) {
    J.hist[i] = 0;
    if (J.phist) J.phist[i] = 0;
  }
  if (threadIdx.x == 0) {
    JobState *st = J.state;
    st->m0 = st->m1 = st->W0 = st->W1 = 0;
    st->status = 0;
    st->tau_key = 0;
    st->cand_count = 0;
    st->nsurv = 0;
    st->l1_count = 0;
    st->l2_count = 0;
    st->kth_key = 0;
    st->flags = 0;
    st->n_sel = 0;
    if (blockIdx.x == 0)
      for (int i = 0; i < kTileCounters; ++i) g.tile_counter[i] = 0;
  }
}

// One workgroup per job: class sizes and the stable class partition
// idx[0..m0) = controls, idx[m0..m) = cases, each in sample order.
__global__ __launch_bounds__(1024) void partition_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.x];
  JobState *st = J.state;
  const uint32_t m = J.m;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ uint32_t s_base1;
  __shared__ uint32_t s_bad;
  if (tid == 0) {
    s_base1 = 0;
    s_bad = 0;
  }
  __syncthreads();
  // pass 1: number of cases
  uint32_t mine = 0;
  for (uint32_t s = tid; s < m; s += blockDim.x) {
    uint8_t v = J.y[s];
    mine += (v == 1);
    if (v > 1) s_bad = 1;
  }
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_down(mine, off);
  if (lane == 0) atomicAdd(&s_base1, mine);
  __syncthreads();
  const uint32_t m1 = s_base1;
  const uint32_t m0 = m - m1;
  if (s_bad) {
    if (tid == 0) st->status = FIUNCHO_E_PHENOTYPE;
    return;
  }
  __syncthreads();
  // pass 2: stable scatter, 4,096 samples per round: thread t takes samples
  // 4t .. 4t + 3 of the round; (controls, cases) counts travel as one u32 of
  // two 16-bit halves through a block-wide exclusive scan
  constexpr uint32_t kPer = 4;
  __shared__ uint32_t s_scan[16];
  uint32_t base0 = 0, base1 = 0;
  for (uint32_t c0 = 0; c0 < m; c0 += kPer * blockDim.x) {
    const uint32_t s0 = c0 + kPer * tid;
    uint32_t cls = 0, cnt = 0;  // bit u of cls: sample s0 + u is a case
#pragma unroll
    for (uint32_t u = 0; u < kPer; ++u) {
      const uint32_t s = s0 + u;
      if (s < m) {
        const bool isc = J.y[s] == 1;
        cls |= (uint32_t)isc << u;
        cnt += isc ? 0x10000u : 1u;
      }
    }
    // inclusive scan over the wave, then over the waves
    uint32_t inc = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)inc, off);
      if (lane >= (uint32_t)off) inc += v;
    }
    if (lane == 63) s_scan[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
      const uint32_t v = s_scan[w];
      if (w < wave) before += v;
      total += v;
    }
    const uint32_t ex = before + inc - cnt;  // this thread's exclusive prefix
    uint32_t p0 = base0 + (ex & 0xFFFFu), p1 = base1 + (ex >> 16);
#pragma unroll
    for (uint32_t u = 0; u < kPer; ++u) {
      const uint32_t s = s0 + u;
      if (s < m) {
        if ((cls >> u) & 1u) J.idx[m0 + p1++] = s;
        else J.idx[p0++] = s;
      }
    }
    base0 += total & 0xFFFFu;
    base1 += total >> 16;
    __syncthreads();
  }
  if (tid == 0) {
    st->m0 = m0;
    st->m1 = m1;
    st->W0 = (m0 + 63) / 64;
    st->W1 = (m1 + 63) / 64;
  }
}

// One wave per (job, variant): builds the three rows of the variant's genotype
// table for both classes, in the two layouts the scan reads, plus the
// per-class genotype counts (the order-1 contingency table).
// Bv[w][j][g] (g = 0, 1) serves lanes that each own a different variant j;
// Bs[j][w][g] (g = 0, 1, 2, then a zero word) serves wave-uniform (scalar)
// reads of one variant.
constexpr int kPackWaves = 8;  // consecutive variants per workgroup

// Words [wb, we) of one class of variant `row`: lane l reads class position
// 64 (w - c0) + l of word w (consecutive lanes read nearby bytes of the row);
// the three genotype ballots of word w go into lane w - blk of b0, b1, b2.
__device__ __forceinline__ void pack_class(const uint8_t *row, const uint32_t *ix, uint32_t c0,
                                           uint32_t size, uint32_t blk, uint32_t wb, uint32_t we,
                                           uint32_t lane,
                                           u64 &b0, u64 &b1, u64 &b2, uint32_t (&cnt)[3],
                                           bool &bad) {
  for (uint32_t w0 = wb; w0 < we; w0 += 8) {
    uint32_t gv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t p = (w0 + u - c0) * 64 + lane;
      const bool valid = w0 + u < we && p < size;
      gv[u] = valid ? (uint32_t)row[ix[p]] : 3u;
      bad |= valid && gv[u] > 2;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (w0 + u >= we) break;
      const u64 x0 = ballot(gv[u] == 0), x1 = ballot(gv[u] == 1), x2 = ballot(gv[u] == 2);
      cnt[0] += popc64(x0);
      cnt[1] += popc64(x1);
      cnt[2] += popc64(x2);
      if (lane == w0 + u - blk) {
        b0 = x0;
        b1 = x1;
        b2 = x2;
      }
    }
  }
}

__global__ __launch_bounds__(kPackWaves * 64) void pack_kernel(Globals g) {
  // one wave per (variant j, block of 64 words): blockIdx.x = group of
  // kPackWaves variants, blockIdx.y = job, blockIdx.z = word block.  The
  // variant-fastest rows (Bv) of the group are staged in LDS and written as
  // 128 contiguous bytes per word.
  __shared__ u64 s_bv[64][2 * kPackWaves + 1];  // padded against bank conflicts
  const JobDesc &J = g.jobs[blockIdx.y];
  const JobState *st = J.state;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = threadIdx.x >> 6;
  const uint32_t j0 = blockIdx.x * kPackWaves;
  const uint32_t j = uni(j0 + wv);
  if (j0 >= J.n_pad) return;  // uniform over the workgroup
  // the status can change while this kernel runs (other workgroups report
  // bad genotypes): one read decides for the whole workgroup
  __shared__ int32_t s_status;
  if (threadIdx.x == 0) s_status = st->status;
  __syncthreads();
  if (s_status != 0) return;
  const uint32_t m0 = st->m0, m1 = st->m1;
  const uint32_t W0 = st->W0, W1 = st->W1, W = W0 + W1;
  const uint32_t wb = blockIdx.z * 64;
  if (wb >= W) return;  // uniform over the workgroup
  const uint32_t we = min(wb + 64, W);
  const uint32_t n_pad = J.n_pad, wcap = J.wcap;
  u64 b0 = 0, b1 = 0, b2 = 0;
  if (j < J.n) {
    // variants j >= n (padding read by the last lanes of a tile) keep zeros
    const uint8_t *row = J.G + (size_t)j * J.m;
    uint32_t cnt[2][3] = {{0, 0, 0}, {0, 0, 0}};
    bool bad = false;
    if (wb < W0) pack_class(row, J.idx, 0, m0, wb, wb, min(we, W0), lane, b0, b1, b2, cnt[0], bad);
    if (we > W0)
      pack_class(row, J.idx + m0, W0, m1, wb, max(wb, W0), we, lane, b0, b1, b2, cnt[1], bad);
    const uint32_t wl = wb + lane;
    if (wl < we) {
      u64 *bs = J.Bs + ((size_t)j * wcap + wl) * 4;
      bs[0] = b0;
      bs[1] = b1;
      bs[2] = b2;
      bs[3] = 0;
    }
    if (ballot(bad)) {
      if (lane == 0) atomicMin(&J.state->status, (int32_t)FIUNCHO_E_GENOTYPE);
    }
    // class counts of this word block; init_kernel cleared them
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int gg = 0; gg < 3; ++gg)
          if (cnt[c][gg]) atomicAdd(&J.marg[((size_t)j * 3 + gg) * 2 + c], cnt[c][gg]);
    }
  }
  s_bv[lane][2 * wv] = b0;
  s_bv[lane][2 * wv + 1] = b1;
  __syncthreads();
  // thread t writes word wb + t / (2 kPackWaves), variant t / 2 mod kPackWaves, plane t mod 2
  for (uint32_t t = threadIdx.x; t < 64 * kPackWaves * 2; t += blockDim.x) {
    const uint32_t ww = t / (2 * kPackWaves), vv = (t / 2) % kPackWaves, gp = t & 1;
    if (wb + ww < we && j0 + vv < n_pad)
      J.Bv[((size_t)(wb + ww) * n_pad + j0 + vv) * 2 + gp] = s_bv[ww][2 * vv + gp];
  }
}

void launch_init(const Globals &g, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(g.n_jobs, kInitBlocks), dim3(256), 0, s, g);
  hipLaunchKernelGGL(partition_kernel, dim3(g.n_jobs), dim3(1024), 0, s, g);
}

void launch_pack(const Globals &g, uint32_t max_n_pad, uint32_t max_wcap, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3((max_n_pad + kPackWaves - 1) / kPackWaves, g.n_jobs, (max_wcap + 63) / 64),
                     dim3(kPackWaves * 64), 0, s, g);
}

}  // namespace fiuncho
