// Per-step kernels of the randomized Arnoldi cycle (Algorithm 1, window-truncated) and of the
// classical Arnoldi comparator, for gfx950.
//
//   k_spmv_sketch : z = A w_j (CSR, one row per lane) fused with u = S z, the sparse-sign sketch
//                   (the product and sketch of Algorithm 1).  S's rows and signs are regenerated
//                   per row from its counter-based specification and scattered into LDS bins, one
//                   set per wavefront; each block writes its partial sketch to the partial buffer.
//                   Batches: one member per block (k_spmv_sketch), or groups of 4, 8 or 16
//                   members per block sharing the staged CSR chunk and the generated rows of S
//                   (k_spmv_sketch_grp).
//   k_reduce_parts: the per-block partials summed in a fixed order (the sketch of z, the norms of
//                   the pass): bit-for-bit the same result on every run.
//   k_orth_update : one launch for step j's Gram-Schmidt and window update (single solves with a
//                   small sketch): persistent blocks, each redoing the sketch-space Gram-Schmidt
//                   in one wavefront while four stream the basis update.
//   k_orth        : one wavefront; modified Gram-Schmidt of the sketch against the last k sketched
//                   basis vectors, the Hessenberg column, rho and the breakdown test.
//   k_update      : w_{j+1} = (z - sum_i r_ij w_i) / rho over the window (the basis update of Algorithm 1).
//   k_gram / k_cgs_update / k_plain_finish : classical Gram-Schmidt applied twice (CGS2) for the
//                   plain restarted Arnoldi comparator.
#include "fab_internal.h"

#include <hip/hip_ext.h>

namespace fab {

// Row tile of a block: blocks are dealt round-robin to the 8 XCDs, so block b runs on XCD b % 8.
// Each XCD gets a contiguous slab of tiles, keeping the stencil neighbours of its rows in its L2.
struct TileWalk {
  int per_xcd, xcd, local, nloc;
  __device__ TileWalk(int ntiles) {
    per_xcd = (ntiles + kXcds - 1) / kXcds;
    xcd = blockIdx.x % kXcds;
    local = blockIdx.x / kXcds;
    nloc = gridDim.x / kXcds;
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; every thread gets the result.  `buf` holds >= 2 * (kThreads/64) doubles and
// `phase` alternates between calls so one barrier per call suffices.
__device__ __forceinline__ double block_sum(double v, double* buf, int& phase) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* b = buf + phase * (kThreads / 64);
  if ((threadIdx.x & 63) == 0) b[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += b[q];
  phase ^= 1;
  return s;
}

// ---------------------------------------------------------------------------------------------
// MODE 0: y = A x and sketch of y;  MODE 1: sketch of x only;  MODE 2: y = A x only.
//
// Each block walks row tiles of kThreads rows (XCD-contiguous slabs).  The tile's nonzeros are
// staged through LDS in chunks of kChunk with coalesced loads of values and column indices (16-byte
// loads from the chunk start rounded down, where the arrays are 16-byte aligned: 3 - 4% on the
// 256^3 operator, 1% on 128^3; element loads otherwise), then
// every lane forms its own row (so stencil gathers of x stay coalesced across the wavefront).
// The sketch of the row value is scattered into FP64 LDS bins, one set per wavefront: a
// wavefront's LDS atomics are applied in one order (its instructions in program order, the lanes of
// one instruction in the hardware's fixed order), so only the four sets are added at the end, in a
// fixed order, into the block's partial in the partial buffer (see part_index; k_reduce_parts adds
// the blocks).  Shared bins would take the wavefronts' adds in whatever order they arrive, and the
// sketch, hence every later step, would change in its last bits from run to run.  The rows and signs of S are regenerated from
// the counter-based specification for every row (no bytes of S are read): with the LDS-staged
// product the generator's integer work overlaps the memory traffic.
// Rows are summed in FP64 for FP32 data too: a stencil row's terms are ~|w|/h^2 while the row sum
// of a smooth w is ~lambda_min |w|, so FP32 sums would lose log10(kappa) digits on exactly the
// slowly converging components; products of FP32 values are exact in FP64, and only the stored z
// is rounded to FP32.
// The product z is stored with the default cache policy: the window update reads it right after.
// With 16-bit column offsets the CSR arrays of the 128^3 operator take 154 MB of the 256 MB
// memory-side cache, which leaves room for z (non-temporal stores measured 2% slower per solve).
// ---------------------------------------------------------------------------------------------
constexpr int kChunk = 2048;
constexpr int kGather = 8;

// Stage nonzeros [cs, cs+len) of the tile into LDS (values and column indices).  All loads are
// issued before the first LDS write, so the tile waits for one memory round trip rather than one
// per element.  Barriers on both sides (the previous chunk has been consumed; this one is ready).
// With colrel (operators whose columns all lie within 16 bits of their tile's first row, row0) the
// columns are read as those 16-bit offsets: 2 bytes per nonzero instead of 4.  Each offset is held
// in a 32-bit register (packed pairs would make every load wait for the previous one).  With sc16
// the offsets are stored in LDS as they are (the reader adds row0), else widened to columns.
template <typename T>
__device__ __forceinline__ void stage_chunk(const T* __restrict__ vals, const int* __restrict__ colind,
                                            const int16_t* __restrict__ colrel, int row0, int cs, int len, T* sv,
                                            int* sc, int16_t* sc16 = nullptr) {
  __syncthreads();
  T tv[kChunk / kThreads];
  if (colrel) {  // uniform over the grid
    int tr[kChunk / kThreads];  // one register per offset: 16-bit pairs would make each load wait
#pragma unroll
    for (int q = 0; q < kChunk / kThreads; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < len) {
        tv[q] = vals[cs + e];
        tr[q] = colrel[cs + e];
      }
    }
#pragma unroll
    for (int q = 0; q < kChunk / kThreads; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < len) {
        sv[e] = tv[q];
        if (sc16) sc16[e] = (int16_t)tr[q];
        else sc[e] = row0 + (int)tr[q];
      }
    }
  } else {
    int tc[kChunk / kThreads];
#pragma unroll
    for (int q = 0; q < kChunk / kThreads; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < len) {
        tv[q] = vals[cs + e];
        tc[q] = colind[cs + e];
      }
    }
#pragma unroll
    for (int q = 0; q < kChunk / kThreads; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < len) {
        sv[e] = tv[q];
        sc[e] = tc[q];
      }
    }
  }
  __syncthreads();
}

// Vectorized staging for 32-bit columns: nonzeros [a0, p1) with a0 = p0 rounded down to 4, in
// 16-byte loads (4 columns, 4 FP32 or 2 x 2 FP64 values per load), stored at LDS position
// index - a0; a load that would pass nnz falls back to element loads.  Positions below p0 - a0 and
// from p1 - a0 on hold neighbours' entries that no row of the tile reads.
template <typename T>
__device__ __forceinline__ void stage_chunk_vec(const T* __restrict__ vals, const int* __restrict__ colind,
                                                int a0, int p1, int nnz, T* sv, int* sc) {
  __syncthreads();
  constexpr int G = kChunk / (4 * kThreads);  // 16-byte groups per thread
  typedef int i4 __attribute__((ext_vector_type(4)));
  typedef T t4 __attribute__((ext_vector_type(4)));
  i4 cv[G];
  t4 vv[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int s0 = a0 + 4 * ((int)threadIdx.x + q * kThreads);
    if (s0 < p1) {
      if (s0 + 4 <= nnz) {
        cv[q] = *reinterpret_cast<const i4*>(colind + s0);
        vv[q] = *reinterpret_cast<const t4*>(vals + s0);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          cv[q][u] = (s0 + u < nnz) ? colind[s0 + u] : 0;
          vv[q][u] = (s0 + u < nnz) ? vals[s0 + u] : T(0);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int e = 4 * ((int)threadIdx.x + q * kThreads);
    if (a0 + e < p1) {
      *reinterpret_cast<i4*>(sc + e) = cv[q];
      *reinterpret_cast<t4*>(sv + e) = vv[q];
    }
  }
  __syncthreads();
}

// The same for 16-bit tile offsets: nonzeros [a0, p1) with a0 = p0 rounded down to 8, 8 offsets
// per 16-byte load and the values in 16-byte loads, the offsets kept as 16 bits in LDS.
template <typename T>
__device__ __forceinline__ void stage_chunk_vec16(const T* __restrict__ vals, const int16_t* __restrict__ colrel,
                                                  int a0, int p1, int nnz, T* sv, int16_t* sc16) {
  __syncthreads();
  constexpr int G = kChunk / (8 * kThreads);  // 8-entry groups per thread
  typedef short s8 __attribute__((ext_vector_type(8)));
  typedef T t8 __attribute__((ext_vector_type(8)));
  s8 cv[G];
  t8 vv[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int s0 = a0 + 8 * ((int)threadIdx.x + q * kThreads);
    if (s0 < p1) {
      if (s0 + 8 <= nnz) {
        cv[q] = *reinterpret_cast<const s8*>(colrel + s0);
        vv[q] = *reinterpret_cast<const t8*>(vals + s0);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          cv[q][u] = (s0 + u < nnz) ? colrel[s0 + u] : (short)0;
          vv[q][u] = (s0 + u < nnz) ? vals[s0 + u] : T(0);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int e = 8 * ((int)threadIdx.x + q * kThreads);
    if (a0 + e < p1) {
      *reinterpret_cast<s8*>(sc16 + e) = cv[q];
      *reinterpret_cast<t8*>(sv + e) = vv[q];
    }
  }
  __syncthreads();
}

// acc + sum of the row's entries [lo, hi) (LDS positions relative to cs) times x, in entry order,
// kGather gathers of x in flight at a time.  Columns from sc (I = int) or as 16-bit offsets from
// the tile's first row row0 (I = int16_t).
template <typename T, typename I>
__device__ __forceinline__ double row_dot(const T* sv, const I* sc, int row0, const T* __restrict__ x, int lo, int hi,
                                          int cs, double acc) {
  for (int pg = lo; pg < hi; pg += kGather) {
    T av[kGather], xv[kGather];
#pragma unroll
    for (int q = 0; q < kGather; ++q) {
      const int p = pg + q;
      av[q] = T(0);
      xv[q] = T(0);
      if (p < hi) {
        av[q] = sv[p - cs];
        xv[q] = x[(sizeof(I) == 2 ? row0 : 0) + (int)sc[p - cs]];
      }
    }
#pragma unroll
    for (int q = 0; q < kGather; ++q) acc = fma((double)av[q], (double)xv[q], acc);
  }
  return acc;
}

// LDS layout of the fused kernel, one member per block: bins (one set of d FP64 per wavefront), then
// the CSR chunk (kChunk values, then kChunk column indices: 16-bit tile offsets on an operator that
// has them, else 32-bit columns).
constexpr int kWaves = kThreads / 64;
__host__ __device__ inline size_t spmv_lds_bins(int mode, int d) {
  return (mode == 2) ? 0 : (((size_t)kWaves * d * 8 + 15) & ~(size_t)15);
}

// row_dot for MU batch members at once (the same row, entries and values, MU vectors): all
// MU x kGather gathers are issued before the first product, so a group of members costs one
// memory round trip per pass instead of one per member.  Members with xs[u] == nullptr are skipped.
template <typename T, int MU>
__device__ __forceinline__ void row_dot_multi(const T* sv, const int* sc, const T* const* xs, int lo, int hi, int cs,
                                              double* acc) {
  for (int pg = lo; pg < hi; pg += kGather) {
    T av[kGather];
    int cv[kGather];
#pragma unroll
    for (int q = 0; q < kGather; ++q) {
      const int p = pg + q;
      av[q] = (p < hi) ? sv[p - cs] : T(0);
      cv[q] = (p < hi) ? sc[p - cs] : -1;
    }
    T xv[MU][kGather];
#pragma unroll
    for (int u = 0; u < MU; ++u)
#pragma unroll
      for (int q = 0; q < kGather; ++q) xv[u][q] = (xs[u] != nullptr && cv[q] >= 0) ? xs[u][cv[q]] : T(0);
#pragma unroll
    for (int u = 0; u < MU; ++u)
#pragma unroll
      for (int q = 0; q < kGather; ++q) acc[u] = fma((double)av[q], (double)xv[u][q], acc[u]);
  }
}

// Occupancy hint of the one-member kernel: for FP32 data at least 8 waves per SIMD (the register
// budget then fits 8 blocks per CU; LDS allows it, and the 256^3 FP32 product runs 17% faster than
// at the default 7).  FP64 blocks that stage 16-bit column offsets: 6 waves (LDS fits 6 blocks of
// 27 KB at d = 200; unhinted, the compiler takes 89 VGPRs, 5 waves).  Other FP64 blocks are limited
// to 5 per CU by LDS anyway: no hint.
template <typename T, bool C16>
constexpr int spmv_min_waves() {
  return sizeof(T) == 4 ? 8 : (C16 ? 6 : 1);
}

// C16: the CSR chunk's columns are staged in LDS as the operator's 16-bit tile offsets (a separate
// instantiation, since one kernel holding both forms needs 101 instead of 75 VGPRs and drops from
// 6 to 4 waves per SIMD).
template <typename T, int MODE, int ZMAX, bool C16 = false>
__global__ __launch_bounds__(kThreads, (spmv_min_waves<T, C16>())) void k_spmv_sketch(int n, const int* __restrict__ rowptr,
                                                          const int* __restrict__ colind,
                                                          const int16_t* __restrict__ colrel,
                                                          const T* __restrict__ vals,
                                                          const T* __restrict__ x, T* __restrict__ y,
                                                          int d, int zeta, T scale, uint32_t k0, uint32_t k1,
                                                          double* __restrict__ parts,
                                                          const State* __restrict__ st, size_t bs, int nts) {
  extern __shared__ unsigned char smem_raw[];
  // This block serves batch member blockIdx.y (0 for single solves).  nts: store z non-temporal
  // (operators whose CSR arrays exceed the memory-side cache; see k_orth_update).
  const int r0 = blockIdx.y;
  {
    const State* sg = st ? bat(st, bs, r0) : nullptr;
    if (sg && (sg->brk || sg->done)) return;  // uniform over the block
  }
  const size_t o_chk = spmv_lds_bins(MODE, d);
  double* bins = reinterpret_cast<double*>(smem_raw);
  T* sv = reinterpret_cast<T*>(smem_raw + o_chk);
  int* sc = reinterpret_cast<int*>(smem_raw + o_chk + kChunk * sizeof(T));
  int16_t* sc16 = C16 ? reinterpret_cast<int16_t*>(sc) : nullptr;
  double* wbins = bins + (threadIdx.x >> 6) * d;  // this wavefront's set
  if (MODE != 2) {
    for (int i = threadIdx.x; i < kWaves * d; i += kThreads) bins[i] = 0.0;
    __syncthreads();
  }
  const T* xg = bat(x, bs, r0);
  // 16-byte staging loads where the CSR arrays allow them (uniform over the grid)
  const bool vec_ok = MODE != 1 && ((((uintptr_t)vals) | ((uintptr_t)(C16 ? (const void*)colrel : (const void*)colind))) & 15) == 0;
  const int nnz_all = vec_ok ? rowptr[n] : 0;
  const int ntiles = (n + kThreads - 1) / kThreads;
  TileWalk tw(ntiles);
  for (int tt = tw.local; tt < tw.per_xcd; tt += tw.nloc) {
    const int tile = tw.xcd * tw.per_xcd + tt;
    if (tile >= ntiles) break;  // uniform over the block
    const int row0 = tile * kThreads;
    const int row = row0 + threadIdx.x;
    const bool live = row < n;
    int p0 = 0, p1 = 0, my_lo = 0, my_hi = 0, a0 = 0;
    bool one_chunk = true;
    if (MODE != 1) {
      const int rend = min(row0 + kThreads, n);
      p0 = rowptr[row0];
      p1 = rowptr[rend];
      my_lo = live ? rowptr[row] : 0;
      my_hi = live ? rowptr[row + 1] : 0;
      a0 = vec_ok ? (p0 & (C16 ? ~7 : ~3)) : p0;
      one_chunk = (p1 - a0) <= kChunk;
      // Wave priority: the tile's loads (CSR chunk, then the row gathers) at a raised priority,
      // the sketch arithmetic at the default one, so the sequencer issues the memory work of the
      // waiting waves first and the ALU work of the sketch fills the gaps between (159 against
      // 153.5 solves/s on the 128^3 workload; the fused kernel 38.7 against 41.0 us)
      __builtin_amdgcn_s_setprio(2);
      if (one_chunk) {
        if (!vec_ok) stage_chunk(vals, colind, colrel, row0, p0, p1 - p0, sv, sc, sc16);
        else if constexpr (C16) stage_chunk_vec16(vals, colrel, a0, p1, nnz_all, sv, sc16);
        else stage_chunk_vec(vals, colind, a0, p1, nnz_all, sv, sc);
      }
    }
    T z = T(0);
    if (MODE != 1) {
      double acc = 0.0;  // FP64 row sums for either value type (see the note above)
      if (one_chunk) {
        if constexpr (C16) acc = row_dot(sv, sc16, row0, xg, my_lo, my_hi, a0, acc);
        else acc = row_dot(sv, sc, row0, xg, my_lo, my_hi, a0, acc);
      } else {  // a tile with more than kChunk nonzeros: stream it through LDS chunk by chunk
        for (int cs = p0; cs < p1; cs += kChunk) {
          const int len = min(kChunk, p1 - cs);
          stage_chunk(vals, colind, colrel, row0, cs, len, sv, sc, sc16);
          if constexpr (C16) acc = row_dot(sv, sc16, row0, xg, max(my_lo, cs), min(my_hi, cs + len), cs, acc);
          else acc = row_dot(sv, sc, row0, xg, max(my_lo, cs), min(my_hi, cs + len), cs, acc);
        }
      }
      z = (T)acc;
      if (live) {
        if (nts) __builtin_nontemporal_store(z, bat(y, bs, r0) + row);
        else bat(y, bs, r0)[row] = z;
      }
    } else if (live) {
      z = xg[row];
    }
    if (MODE != 2 && live) {  // scatter straight from the row's lane
      int rows[ZMAX];
      uint32_t sb = 0;
      __builtin_amdgcn_s_setprio(0);
      sketch_column<ZMAX>((uint64_t)row, d, zeta, k0, k1, rows, sb);
      const double zs = (double)z * (double)scale;
#pragma unroll
      for (int l = 0; l < ZMAX; ++l)
        if (l < zeta) unsafeAtomicAdd(&wbins[rows[l]], ((sb >> l) & 1u) ? -zs : zs);
    }
  }
  if (MODE != 2) {  // the block's partial sketch, the wavefront sets added in a fixed order
    __syncthreads();
    const size_t pidx = part_index();
    double* pg = bat(parts, bs, r0);
    for (int b = threadIdx.x; b < d; b += kThreads) {
      double v = bins[b];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) v += bins[w * d + b];
      pg[(size_t)b * kMaxParts + pidx] = v;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Batch members in groups of G (4, 8 or 16) per block: the tile's CSR chunk is staged once and
// applied to every member's vector, and the rows and signs of S are generated once per row, into
// an LDS table, while the chunk's loads are in flight.  Wavefront w then owns members
// w G/4 .. (w+1) G/4 - 1 over all rows of the tile (lane = row, 64 rows at a time, so the gathers
// of each member stay coalesced) and scatters their rows of the sketch into one FP64 bin set per
// block, laid out [member][bin]: every (member, bin) entry has a single writer wavefront, whose
// LDS atomics apply in program order (and in the hardware's fixed lane order within one
// instruction), so the block's partial is the same on every run.  S is sparse (zeta of d entries
// per column): the scatter does zeta updates per row and member, where a dense contraction on the
// matrix cores would multiply by d - zeta zeros.
// LDS: bins (G d FP64), the tile's table (ZMAX 16-bit rows and a 32-bit sign word per row), then
// (products) the CSR chunk with 32-bit columns.
// ---------------------------------------------------------------------------------------------
constexpr int kGroupMax = 16;                    // largest group (4 members per wavefront)
constexpr int kWaveMembers = kGroupMax / kWaves;  // members a wavefront owns at most

__host__ __device__ inline size_t grp_lds_bins(int d, int G) { return ((size_t)G * d * 8 + 15) & ~(size_t)15; }
__host__ __device__ inline size_t grp_lds_table(int zmax) {
  return ((size_t)kThreads * (2 * zmax + 4) + 15) & ~(size_t)15;
}

// Occupancy hint: 4 waves per SIMD, whose 128 registers hold the gathers of four FP32 members
// (two FP64) in flight without spilling; at 5 (the most LDS allows for FP32 blocks at d = 80) the
// FP32 kernel spills.
template <typename T>
constexpr int grp_min_waves() {
  return sizeof(T) == 4 ? 5 : 4;
}

// Buffer resources and loads (defined with the window update below).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, int bytes);
template <int AUX>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int off, double);
template <int AUX>
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int off, float);

// row_dot for the NM members a wavefront owns in the grouped kernel (NM = G / 4).  Each pass reads
// its kGather LDS entries once (entries past the row's end read its last entry, with value 0 and
// the byte offset `end`, one past every member's buffer) and forms their byte offsets once; every
// member's gathers are then buffer loads at those offsets (member u's x as a buffer of `end` bytes,
// of 0 bytes for a member that has finished), with no address arithmetic and no branch per member,
// two members' gathers issued before their products.  Out-of-range loads return 0 without
// touching memory.  Per member the sums are row_dot's: entries in order, FP64 fma.  The buffer
// resources are formed at each use: held across the kernel, their scalar registers pushed other
// values into vector registers, and those into scratch.
template <typename T, int NM>
__device__ __forceinline__ void row_dot_members(const T* sv, const int* sc, const T* const (&xs)[kWaveMembers],
                                                const bool (&own)[kWaveMembers], int lo, int hi, int cs, int end,
                                                double (&acc)[kWaveMembers]) {
  constexpr int MF = NM < 2 ? NM : 2;  // members in flight: four FP32 members' gathers spill at 5 waves
  for (int pg = lo; pg < hi; pg += kGather) {
    T av[kGather];
    int bo[kGather];
#pragma unroll
    for (int q = 0; q < kGather; ++q) {
      const int p = pg + q;
      const int pc = min(p, hi - 1) - cs;  // an entry of this row in the chunk (pg < hi)
      const T a = sv[pc];
      const int c = sc[pc];
      av[q] = (p < hi) ? a : T(0);
      bo[q] = (p < hi) ? c * (int)sizeof(T) : end;
    }
#pragma unroll
    for (int u0 = 0; u0 < NM; u0 += MF) {
      T xv[MF][kGather];
#pragma unroll
      for (int v = 0; v < MF; ++v) {
        const __amdgpu_buffer_rsrc_t rx = buf_rsrc(xs[u0 + v], own[u0 + v] ? end : 0);
#pragma unroll
        for (int q = 0; q < kGather; ++q) xv[v][q] = buf_load<0>(rx, bo[q], T());
      }
#pragma unroll
      for (int v = 0; v < MF; ++v)
#pragma unroll
        for (int q = 0; q < kGather; ++q) acc[u0 + v] = fma((double)av[q], (double)xv[v][q], acc[u0 + v]);
    }
  }
}

template <typename T, int MODE, int ZMAX>
__global__ __launch_bounds__(kThreads, (grp_min_waves<T>())) void k_spmv_sketch_grp(int n, const int* __restrict__ rowptr,
                                                              const int* __restrict__ colind,
                                                              const int16_t* __restrict__ colrel,
                                                              const T* __restrict__ vals,
                                                              const T* __restrict__ x, T* __restrict__ y, int d,
                                                              int zeta, T scale, uint32_t k0, uint32_t k1,
                                                              double* __restrict__ parts,
                                                              const State* __restrict__ st, int nb, int G,
                                                              size_t bs) {
  static_assert(MODE == 0 || MODE == 1, "the grouped kernel forms sketches");
  extern __shared__ unsigned char smem_raw[];
  const int r0 = blockIdx.y * G;
  const int gn = min(G, nb - r0);
  uint32_t live_mask = 0;  // members still iterating (block-uniform)
  for (int g = 0; g < gn; ++g) {
    const State* sg = st ? bat(st, bs, r0 + g) : nullptr;
    if (!sg || !(sg->brk || sg->done)) live_mask |= 1u << g;
  }
  if (live_mask == 0) return;
  const size_t o_tab = grp_lds_bins(d, G);
  const size_t o_chk = o_tab + grp_lds_table(ZMAX);
  double* bins = reinterpret_cast<double*>(smem_raw);                       // [member][bin]
  uint16_t* trow = reinterpret_cast<uint16_t*>(smem_raw + o_tab);           // [row][ZMAX]
  uint32_t* tsgn = reinterpret_cast<uint32_t*>(trow + kThreads * ZMAX);     // [row]
  T* sv = reinterpret_cast<T*>(smem_raw + o_chk);
  int* sc = reinterpret_cast<int*>(smem_raw + o_chk + kChunk * sizeof(T));
  for (int i = threadIdx.x; i < G * d; i += kThreads) bins[i] = 0.0;
  // the wavefront index as a scalar: the member pointers below then live in scalar registers and
  // the per-member branches are scalar branches
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int per_wave = G / kWaves;
  // Every member pointer is a real member's (the block's first when the slot is not owned), so the
  // compiler keeps them in the global address space: a null among them made the gathers flat loads,
  // which also count against the LDS wait counter (global loads: 577 -> 567 us per launch on 64
  // FP32 members of 1024^2).
  const T* xs[kWaveMembers];
  T* ys[kWaveMembers];
  int gs[kWaveMembers];
  bool own[kWaveMembers];
#pragma unroll
  for (int u = 0; u < kWaveMembers; ++u) {
    const int g = wv * per_wave + u;
    own[u] = u < per_wave && g < gn && ((live_mask >> g) & 1u);
    gs[u] = g;
    xs[u] = bat(x, bs, r0 + (own[u] ? g : 0));
    ys[u] = bat(y, bs, r0 + (own[u] ? g : 0));
  }
  const double dscale = (double)scale;
  const int ntiles = (n + kThreads - 1) / kThreads;
  TileWalk tw(ntiles);
  for (int tt = tw.local; tt < tw.per_xcd; tt += tw.nloc) {
    const int tile = tw.xcd * tw.per_xcd + tt;
    if (tile >= ntiles) break;  // uniform over the block
    const int row0 = tile * kThreads;
    int p0 = 0, p1 = 0;
    bool one_chunk = true;
    if (MODE == 0) {
      p0 = rowptr[row0];
      p1 = rowptr[min(row0 + kThreads, n)];
      one_chunk = (p1 - p0) <= kChunk;
    }
    __syncthreads();  // the previous tile's chunk and table have been read (and the bins zeroed)
    // The tile's CSR chunk staged in LDS and the table rows of S generated.  FP64: the table while
    // the chunk's loads are in flight.  FP32 (whose row loop holds more registers): the chunk in two
    // halves, then the table; staged whole, with the table in between, the loaded values were
    // spilled to scratch one load at a time.
    {
      constexpr int kParts = sizeof(T) == 4 ? 2 : 1;
      constexpr int kPer = kChunk / kThreads / kParts;
      const bool stage = MODE == 0 && one_chunk;
      auto gen_table = [&]() {
        const int row = row0 + threadIdx.x;
        int rows[ZMAX];
        uint32_t sb = 0;
        if (row < n) sketch_column<ZMAX>((uint64_t)row, d, zeta, k0, k1, rows, sb);
#pragma unroll
        for (int l = 0; l < ZMAX; ++l) trow[threadIdx.x * ZMAX + l] = (row < n) ? (uint16_t)rows[l] : (uint16_t)0;
        tsgn[threadIdx.x] = sb;
      };
#pragma unroll
      for (int h = 0; h < kParts; ++h) {
        T tv[kPer];
        int tc[kPer];
        if (stage) {
#pragma unroll
          for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + (h * kPer + q) * kThreads;
            if (e < p1 - p0) {
              tv[q] = vals[p0 + e];
              tc[q] = colrel ? row0 + (int)colrel[p0 + e] : colind[p0 + e];
            }
          }
        }
        if (sizeof(T) == 8) gen_table();
        if (stage) {
#pragma unroll
          for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + (h * kPer + q) * kThreads;
            if (e < p1 - p0) {
              sv[e] = tv[q];
              sc[e] = tc[q];
            }
          }
        }
      }
      if (sizeof(T) == 4) gen_table();
    }
    __syncthreads();
#pragma unroll 1
    for (int rg = 0; rg < kWaves; ++rg) {  // uniform over the block
      const int lr = rg * 64 + lane;
      const int row = row0 + lr;
      const bool live = row < n;
      double acc[kWaveMembers];
#pragma unroll
      for (int u = 0; u < kWaveMembers; ++u) acc[u] = 0.0;
      if (MODE == 0) {
        const int lo = live ? rowptr[row] : 0, hi = live ? rowptr[row + 1] : 0;
        // the shared gathers for FP32 values and tables of up to 8 rows: wider tables leave no
        // registers for them, and the FP64 instantiations keep the previous form (with the shared
        // gathers, the scatter below and the staging above they measured 7 - 10% slower on 16 and
        // on 4 FP64 members of 512^2)
        if (one_chunk && (ZMAX > 8 || sizeof(T) == 8)) {
#pragma unroll
          for (int u = 0; u < kWaveMembers; ++u)
            if (own[u]) acc[u] = row_dot(sv, sc, 0, xs[u], lo, hi, p0, 0.0);
        } else if (one_chunk) {
          const int end = n * (int)sizeof(T);
          if (per_wave == 4)  // uniform over the block
            row_dot_members<T, 4>(sv, sc, xs, own, lo, hi, p0, end, acc);
          else if (per_wave == 2)
            row_dot_members<T, 2>(sv, sc, xs, own, lo, hi, p0, end, acc);
          else
            row_dot_members<T, 1>(sv, sc, xs, own, lo, hi, p0, end, acc);
        } else {  // a tile with more than kChunk nonzeros: its chunks in turn, for this row group
          for (int cs = p0; cs < p1; cs += kChunk) {
            const int len = min(kChunk, p1 - cs);
            stage_chunk(vals, colind, colrel, row0, cs, len, sv, sc);
#pragma unroll
            for (int u = 0; u < kWaveMembers; ++u)
              if (own[u]) acc[u] = row_dot(sv, sc, 0, xs[u], max(lo, cs), min(hi, cs + len), cs, acc[u]);
          }
        }
      } else if (live) {
#pragma unroll
        for (int u = 0; u < kWaveMembers; ++u)
          if (own[u]) acc[u] = (double)xs[u][row];
      }
      if (live) {
        // FP32 values and tables of up to 8 rows: the row's bin offsets and sign bits formed once
        // for all members and before the member branches (formed inside them, every branch join
        // waited for the table's LDS reads again, and with them for all scatter atomics issued so
        // far).  Wider tables would spill their 2 ZMAX registers; FP64 keeps the previous form.
        if (ZMAX <= 8 && sizeof(T) == 4) {
          constexpr int ZH = ZMAX <= 8 ? ZMAX : 1;
          uint32_t boff[ZH], sgn[ZH];
          const uint32_t sb = tsgn[lr];
#pragma unroll
          for (int l = 0; l < ZH; ++l) {
            boff[l] = (uint32_t)trow[lr * ZMAX + l] * 8u;
            sgn[l] = ((sb >> l) & 1u) << 31;
          }
#pragma unroll
          for (int u = 0; u < kWaveMembers; ++u) {
            if (!own[u]) continue;  // uniform over the wavefront
            const T z = (T)acc[u];
            if (MODE == 0) ys[u][row] = z;
            const double zs = (double)z * dscale;
            const uint32_t zlo = (uint32_t)__double_as_longlong(zs);
            const uint32_t zhi = (uint32_t)((uint64_t)__double_as_longlong(zs) >> 32);
            unsigned char* mb = reinterpret_cast<unsigned char*>(bins + (size_t)gs[u] * d);
#pragma unroll
            for (int l = 0; l < ZH; ++l)
              if (l < zeta)  // -zs for a set sign bit: the same value as negation
                unsafeAtomicAdd(reinterpret_cast<double*>(mb + boff[l]),
                                __longlong_as_double((long long)(((uint64_t)(zhi ^ sgn[l]) << 32) | zlo)));
          }
        } else {
          uint16_t rows[ZMAX];
#pragma unroll
          for (int l = 0; l < ZMAX; ++l) rows[l] = trow[lr * ZMAX + l];
          const uint32_t sb = tsgn[lr];
#pragma unroll
          for (int u = 0; u < kWaveMembers; ++u) {
            if (!own[u]) continue;  // uniform over the wavefront
            const T z = (T)acc[u];
            if (MODE == 0) ys[u][row] = z;
            const double zs = (double)z * dscale;
            double* mb = bins + (size_t)gs[u] * d;
#pragma unroll
            for (int l = 0; l < ZMAX; ++l)
              if (l < zeta) unsafeAtomicAdd(&mb[rows[l]], ((sb >> l) & 1u) ? -zs : zs);
          }
        }
      }
    }
  }
  __syncthreads();  // the block's partial sketch of every live member
  const size_t pidx = part_index();
  for (int i = threadIdx.x; i < G * d; i += kThreads) {
    const int g = i / d, b = i - g * d;
    if (g >= gn || !((live_mask >> g) & 1u)) continue;
    bat(parts, bs, r0 + g)[(size_t)b * kMaxParts + pidx] = bins[i];
  }
}

// out[i] = sum over p < nparts of parts[(e0 + i) * kMaxParts + p] for i = blockIdx.x, one block per
// entry and member (blockIdx.y), in a fixed order: thread t adds p = t, t + kThreads, ... in turn
// (all its loads issued first), a butterfly sums each wavefront, and the wavefront sums are added in
// order.  Members are skipped as their producer skipped them: skip 0 = broken down or finished (the
// fused product), 1 = finished, non-finite or empty (the pass), -1 = never.
__global__ __launch_bounds__(kThreads) void k_reduce_parts(int e0, int nparts, const double* __restrict__ parts,
                                                           double* __restrict__ out, const State* __restrict__ st,
                                                           int skip, size_t bs) {
  __shared__ double ws[kWaves];
  if (st && skip >= 0) {
    const State* sm = bat(st, bs);
    if (skip == 0 ? (sm->brk || sm->done) : (sm->done || sm->nonfinite || sm->meff == 0)) return;
  }
  const double* src = bat(parts, bs) + (size_t)(e0 + (int)blockIdx.x) * kMaxParts;
  double v[kMaxParts / kThreads];
#pragma unroll
  for (int u = 0; u < kMaxParts / kThreads; ++u) {
    const int p = threadIdx.x + u * kThreads;
    v[u] = (p < nparts) ? src[p] : 0.0;
  }
  double s = v[0];
#pragma unroll
  for (int u = 1; u < kMaxParts / kThreads; ++u) s += v[u];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = ws[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) r += ws[w];
    bat(out, bs)[blockIdx.x] = r;
  }
}

// ---------------------------------------------------------------------------------------------
// Sketch-space modified Gram-Schmidt of step j, one wavefront (no barriers).  Element e of the
// d-vector lives in lane e % 64, slot e / 64 (PER slots per lane, d <= 64 PER).
// uraw: S z (d values, the fixed-order sum of the product's partials); U: d x (m+1) sketched
// basis.  When `coef` is given, lane 0 stores the window coefficients r_ij there (index i - lo,
// i = lo..j), 1/rho in *inv and the outcome (1 = a new basis vector) in *ok; when `write`, the
// wavefront also stores R column j, U column j+1 and the step's state.
// ---------------------------------------------------------------------------------------------
// KW > 0: the window's KW columns of U are loaded together with S z (one memory round trip
// instead of one per window column; requires j - lo + 1 <= KW).  When `unew` is given, the lanes
// receive their PER entries of u_{j+1} there (unchanged on breakdown).
template <int PER, int KW>
__device__ __forceinline__ void orth_wave(int j, int k, int m, int d, const double* __restrict__ uraw,
                                          double* __restrict__ U, double* __restrict__ R, State* __restrict__ st,
                                          bool write, double* coef, double* inv_out, int* ok_out,
                                          double* unew = nullptr, const double* __restrict__ parts = nullptr,
                                          int nparts = 0) {
  const int lane = threadIdx.x & 63;
  const int lo = max(0, j - k + 1);
  double u[PER];
  double upre[KW > 0 ? KW : 1][PER];
  if (KW > 0) {
#pragma unroll
    for (int w = 0; w < (KW > 0 ? KW : 1); ++w)
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = lane + 64 * q;
        upre[w][q] = (lo + w <= j && e < d) ? U[(size_t)(lo + w) * d + e] : 0.0;
      }
  }
  if (parts == nullptr) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = lane + 64 * q;
      u[q] = (e < d) ? uraw[e] : 0.0;
    }
  } else {
    // S z from the product's per-block partials (small grids, nparts <= 64): each lane adds the
    // partials of its own entries in block order, eight loads in flight (a fixed order: the same
    // bits on every run; not the order of k_reduce_parts)
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = lane + 64 * q;
      double acc = 0.0;
      if (e < d) {
        const double* src = parts + (size_t)e * kMaxParts;
        for (int p0 = 0; p0 < nparts; p0 += 8) {
          double v[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) v[r] = (p0 + r < nparts) ? src[p0 + r] : 0.0;
#pragma unroll
          for (int r = 0; r < 8; ++r) acc += v[r];
        }
      }
      u[q] = acc;
    }
  }
  double loc = 0.0;
#pragma unroll
  for (int q = 0; q < PER; ++q) loc += u[q] * u[q];
  const double raw2 = wave_sum(loc);
  // one modified Gram-Schmidt step against window column i (values ui)
  auto mgs = [&](int i, const double* ui) {
    double l2 = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) l2 += ui[q] * u[q];
    const double r = wave_sum(l2);
#pragma unroll
    for (int q = 0; q < PER; ++q) u[q] -= r * ui[q];
    if (coef && lane == 0) coef[i - lo] = r;
    if (write && lane == 0) {
      R[(size_t)j * (m + 1) + i] = r;
      st->upd_coef[i - lo] = r;
    }
  };
  if constexpr (KW > 0) {
#pragma unroll
    for (int w = 0; w < KW; ++w)
      if (lo + w <= j) mgs(lo + w, upre[w]);
  } else {
    for (int i = lo; i <= j; ++i) {
      const double* Ui = U + (size_t)i * d;
      double ui[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = lane + 64 * q;
        ui[q] = (e < d) ? Ui[e] : 0.0;
      }
      mgs(i, ui);
    }
  }
  loc = 0.0;
#pragma unroll
  for (int q = 0; q < PER; ++q) loc += u[q] * u[q];
  const double rho = sqrt(wave_sum(loc));
  const bool finite = isfinite(rho) && isfinite(raw2);
  const bool breakdown = !(rho > 64.0 * 2.220446049250313e-16 * sqrt(raw2));
  if (!finite || breakdown) {
    if (coef && lane == 0) {
      *ok_out = 0;
      *inv_out = 0.0;
    }
    if (write && lane == 0) {
      st->brk = 1;
      st->meff = j + 1;
      if (!finite) st->nonfinite = 1;
    }
    return;
  }
  const double inv = 1.0 / rho;
  if (coef && lane == 0) {
    *ok_out = 1;
    *inv_out = inv;
  }
  if (unew) {
#pragma unroll
    for (int q = 0; q < PER; ++q) unew[q] = u[q] * inv;
  }
  if (write) {
    double* Un = U + (size_t)(j + 1) * d;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = lane + 64 * q;
      if (e < d) Un[e] = u[q] * inv;
    }
    if (lane == 0) {
      R[(size_t)j * (m + 1) + j + 1] = rho;
      st->inv_rho = inv;
      st->step_lo = lo;
    }
  }
}

template <int PER>
__global__ __launch_bounds__(64) void k_orth(int j, int k, int m, int d, const double* __restrict__ uraw,
                                             double* __restrict__ U, double* __restrict__ R, State* __restrict__ st,
                                             size_t bs) {
  st = bat(st, bs);
  if (st->brk || st->done) return;
  orth_wave<PER, 0>(j, k, m, d, bat(uraw, bs), bat(U, bs), bat(R, bs), st, true, nullptr, nullptr, nullptr);
}

// Step j's Gram-Schmidt and window update in one launch (d <= 256), with persistent blocks.
// Blocks of 1 + 4 wavefronts: the first redoes the sketch-space Gram-Schmidt (the same
// arithmetic on the same S z in every block, so every block gets the same coefficients; block 0 also stores
// R, U and the state) while the other four load their first batch of elements (z and the window).
// After the barrier they stream the block's batches of OuBatch elements, and the loads of the
// next batch are issued before the current one is updated and stored, so reads and writes of the
// whole grid overlap instead of running in two phases.  (A wavefront's loads complete in order, so
// the Gram-Schmidt gets a wavefront of its own: streaming loads issued by the same wavefront would
// hold up its reads of the sketch.)  Load indices are clamped into the vector instead of guarded:
// with no branch around a load, the compiler can count the loads in flight and wait for one batch
// only.  Saves the separate single-wavefront launch, whose latency would sit between product and
// update, and runs the Gram-Schmidt once per block rather than once per 1024 elements.
// Elements per streaming thread and batch: 4, except 2 for FP64 under the non-temporal policy
// (operators beyond the memory-side cache).  Measured against 2 throughout: the 256^3 FP32 step
// 298 -> 290 us (its update had run at 0.66 of peak against 0.77 for FP64), the 128^3 FP64 step
// 53.85 -> 53.27 us; the 256^3 FP64 step 457.9 -> 460.7 us with 4, hence 2 there.
template <typename T, int AUX>
struct OuPer {
  static constexpr int v = (sizeof(T) == 8 && AUX != 0) ? 2 : 4;
};
constexpr int kOuThreads = 64 + kThreads;  // Gram-Schmidt wavefront + streaming wavefronts
template <typename T, int AUX>
struct OuBatch {  // elements per block and batch
  static constexpr int v = kThreads * OuPer<T, AUX>::v;
};
// Blocks per CU: 3 under the default cache policy, 2 under the non-temporal one (measured against
// 2 throughout: the 128^3 FP64 step 53.2 -> 52.6 us with 3, 54.6 with 4; the 256^3 FP64 step
// 458.0 -> 462.5 us with 3).
constexpr int ou_blocks_per_cu(int nts) { return nts ? 2 : 3; }

// Raw buffer accesses (untyped, byte offsets): the hardware checks every lane's offset against the
// resource's size, returns 0 for a load beyond it and drops a store beyond it, so a ragged batch
// needs no branch.  Word 3 of the gfx9-family descriptor: 32-bit data format (a valid format is
// required for untyped accesses), all other fields zero.  The cache policy is the operator's: the
// default one when its CSR arrays fit the 256 MB memory-side cache with room to spare, since the
// new basis vector is gathered by the next step's product and read by the next windows, and z and
// the window columns were written moments ago (non-temporal hints measured 0.5 us per step slower
// on a 154 MB CSR); non-temporal when the CSR arrays stream through that cache anyway, where the
// default policy lets the vectors evict the arrays' lines for nothing (measured 2-3% per cycle
// on a 1.4 GB CSR).
constexpr int kBufWord3 = 0x00020000;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, kBufWord3);
}
// AUX: the cache-policy operand of the access, 0 (default) or kAuxNt (non-temporal).
constexpr int kAuxNt = 2;
template <int AUX>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, AUX);
}
template <int AUX>
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, AUX);
}

// Elements of one batch: those of [b0, b0 + OuBatch) below n (none when b0 >= n: a size-0
// resource, whose loads return 0 without touching memory).
template <typename T, int AUX>
__device__ __forceinline__ int ou_count(int n, int64_t b0) {
  return b0 < n ? (int)min((int64_t)OuBatch<T, AUX>::v, (int64_t)n - b0) : 0;
}

template <typename T, int KMAX, int AUX>
__device__ __forceinline__ void ou_load(const T* __restrict__ out, const T* __restrict__ base, int n, size_t ld,
                                        int nw, int64_t b0, int t, T (&zv)[OuPer<T, AUX>::v], T (&wv)[OuPer<T, AUX>::v][KMAX]) {
  const int cnt = ou_count<T, AUX>(n, b0);
  const int64_t o = cnt ? b0 : 0;
  const __amdgpu_buffer_rsrc_t rz = buf_rsrc(out + o, cnt * (int)sizeof(T));
  __amdgpu_buffer_rsrc_t rw[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q)  // columns beyond the window: size 0 (their coefficients are 0)
    rw[q] = buf_rsrc(base + (size_t)min(q, nw - 1) * ld + o, q < nw ? cnt * (int)sizeof(T) : 0);
#pragma unroll
  for (int e = 0; e < OuPer<T, AUX>::v; ++e) {
    const int off = (e * kThreads + t) * (int)sizeof(T);
    zv[e] = buf_load<AUX>(rz, off, T());
#pragma unroll
    for (int q = 0; q < KMAX; ++q) wv[e][q] = buf_load<AUX>(rw[q], off, T());
  }
}

// FP64 arithmetic for either value type: z is nearly in the span of the window, so the difference
// cancels; only the stored w_{j+1} is rounded to T.  coef is zero beyond the window.
template <typename T, int KMAX, int AUX>
__device__ __forceinline__ void ou_store(T* __restrict__ out, int n, int64_t b0, int t, const double (&coef)[KMAX],
                                         double inv, const T (&zv)[OuPer<T, AUX>::v], const T (&wv)[OuPer<T, AUX>::v][KMAX]) {
  const int cnt = ou_count<T, AUX>(n, b0);
  const __amdgpu_buffer_rsrc_t rz = buf_rsrc(out + (cnt ? b0 : 0), cnt * (int)sizeof(T));
#pragma unroll
  for (int e = 0; e < OuPer<T, AUX>::v; ++e) {
    double v = (double)zv[e];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) v -= coef[q] * (double)wv[e][q];
    buf_store<AUX>((T)(v * inv), rz, (e * kThreads + t) * (int)sizeof(T));
  }
}

// The update's batches after the first: two register sets in turn; the prefetch past the block's
// last batch has size 0 (no memory traffic), so every trip issues the same loads and stores
// (loads at raised wave priority, as in the fused product: measured 0.1 us per step).
template <typename T, int KMAX, int AUX, typename Start>
__device__ __forceinline__ void ou_stream(T* __restrict__ out, const T* __restrict__ base, int n, size_t ld, int nw,
                                          int cnt, Start start, int t, const double (&coef)[KMAX], double inv,
                                          T (&za)[OuPer<T, AUX>::v], T (&wa)[OuPer<T, AUX>::v][KMAX], T (&zb)[OuPer<T, AUX>::v],
                                          T (&wb)[OuPer<T, AUX>::v][KMAX]) {
  for (int it = 0;;) {
    __builtin_amdgcn_s_setprio(2);
    ou_load<T, KMAX, AUX>(out, base, n, ld, nw, start(it + 1), t, zb, wb);
    __builtin_amdgcn_s_setprio(0);
    ou_store<T, KMAX, AUX>(out, n, start(it), t, coef, inv, za, wa);
    if (++it >= cnt) break;
    __builtin_amdgcn_s_setprio(2);
    ou_load<T, KMAX, AUX>(out, base, n, ld, nw, start(it + 1), t, za, wa);
    __builtin_amdgcn_s_setprio(0);
    ou_store<T, KMAX, AUX>(out, n, start(it), t, coef, inv, zb, wb);
    if (++it >= cnt) break;
  }
}

// Row j+1 of the sketched Gram matrix G = U^T U, spread over the blocks of step j's update: entry
// e = 0..j+1 is <u_{j+1}, u_e> (e = j+1: the new vector with itself), and step 0 adds <u_0, u_0>
// as entry 2.  Block b takes entries b, b + gridDim.x, ... in groups of kGramGroup, whose columns
// of U are loaded together, after the barrier that releases the streaming wavefronts (loading them
// before the Gram-Schmidt delays that barrier: measured 0.6 us per step).  The cycle end factors G
// by Cholesky instead of running a Householder QR of U (the whitening), which takes most of that
// work off the path between the last step and the pass.
constexpr int kGramGroup = 2;

__device__ __forceinline__ int gram_entries(int j) { return j + 2 + (j == 0 ? 1 : 0); }

__device__ __forceinline__ void gram_load(const double* __restrict__ U, int d, int j, int e, int lane,
                                          double (&v)[4]) {
  // U column of entry e: e itself for e <= j, column 0 for step 0's extra entry, none otherwise
  const int col = (e <= j) ? e : ((j == 0 && e == 2) ? 0 : -1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    v[q] = (col >= 0 && i < d) ? U[(size_t)col * d + i] : 0.0;
  }
}

// INL: S z summed from the partials (see orth_wave); AUX: the cache policy of the update's loads and
// stores (see buf_rsrc)
template <typename T, int KMAX, bool INL = false, int AUX = 0>
__global__ __launch_bounds__(kOuThreads) void k_orth_update(int n, int j, int k, int m, int d, T* __restrict__ W,
                                                          const double* __restrict__ uraw, double* __restrict__ U,
                                                          double* __restrict__ R, double* __restrict__ G,
                                                          State* __restrict__ st, size_t bs,
                                                          const double* __restrict__ parts, int nparts) {
  __shared__ double s_coef[kMaxM + 1];
  __shared__ double s_inv;
  __shared__ int s_ok;
  st = bat(st, bs);
  if (st->brk || st->done) return;
  W = bat(W, bs);
  const int lo = max(0, j - k + 1), nw = j - lo + 1;
  const size_t ld = wcol(n, sizeof(T));
  T* out = W + (size_t)(j + 1) * ld;
  const T* base = W + (size_t)lo * ld;
  if (threadIdx.x < 64) {
    __builtin_amdgcn_s_setprio(3);  // every wavefront of the block waits for this one at the barrier
    const int lane = threadIdx.x;
    const double* Ub = bat(U, bs);
    const int ne = gram_entries(j);
    double gv[kGramGroup][4], un[4] = {0.0, 0.0, 0.0, 0.0};
    orth_wave<4, KMAX>(j, k, m, d, bat(uraw, bs), bat(U, bs), bat(R, bs), st, blockIdx.x == 0, s_coef, &s_inv,
                       &s_ok, un, INL ? bat(parts, bs) : nullptr, nparts);
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    if (!s_ok) return;  // breakdown: row j+1 does not exist
    double* Gb = bat(G, bs);
    const int ldg = m + 1;
    for (int e0 = (int)blockIdx.x; e0 < ne; e0 += kGramGroup * (int)gridDim.x) {
#pragma unroll
      for (int r = 0; r < kGramGroup; ++r) gram_load(Ub, d, j, e0 + r * (int)gridDim.x, lane, gv[r]);
#pragma unroll
      for (int r = 0; r < kGramGroup; ++r) {
        const int e = e0 + r * (int)gridDim.x;
        if (e >= ne) break;
        const bool self0 = (j == 0 && e == 2);  // <u_0, u_0>
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += (self0 ? gv[r][q] : un[q]) * (e == j + 1 ? un[q] : gv[r][q]);
        const double g = wave_sum(acc);
        if (lane == 0) {
          if (self0) Gb[0] = g;
          else Gb[(size_t)(j + 1) * ldg + e] = g;
        }
      }
    }
    if (blockIdx.x == 0 && lane == 0) st->gram_rows = j + 2;
    return;
  }
  // batches blockIdx.x, blockIdx.x + gridDim.x, ...; the launch keeps gridDim.x <= the batch count
  const int t = threadIdx.x - 64;
  const int nbat = (n + OuBatch<T, AUX>::v - 1) / OuBatch<T, AUX>::v;
  const int cnt = (nbat - 1 - (int)blockIdx.x) / (int)gridDim.x + 1;
  auto start = [&](int it) { return ((int64_t)blockIdx.x + (int64_t)it * gridDim.x) * OuBatch<T, AUX>::v; };
  T za[OuPer<T, AUX>::v], wa[OuPer<T, AUX>::v][KMAX], zb[OuPer<T, AUX>::v], wb[OuPer<T, AUX>::v][KMAX];
  ou_load<T, KMAX, AUX>(out, base, n, ld, nw, start(0), t, za, wa);
  __syncthreads();
  if (!s_ok) return;  // breakdown (or non-finite): the cycle ends at this step
  const double inv = s_inv;
  double coef[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) coef[q] = (q < nw) ? s_coef[q] : 0.0;
  ou_stream<T, KMAX, AUX>(out, base, n, ld, nw, cnt, start, t, coef, inv, za, wa, zb, wb);
}

// w_{j+1} = (z - sum_{i=lo..j} r_i w_i) / rho, in place on column j+1 of W (n x (m+1)).
// KMAX bounds the window so the coefficients live in registers.  Streaming loads and stores are
// non-temporal: a batch's basis columns exceed the memory-side cache many times over.  Each thread
// takes 16 bytes of every column at once (4 FP32 or 2 FP64 values: columns start on 4 KB pages, so
// the vectors are aligned), the last n mod that count elements one by one; per element the
// arithmetic and its order are those of one element at a time, so the bits do not depend on it
// (FP32, 64 members of 1024^2: 279 -> 158 us per launch in the trace, 0.85 of HBM peak).
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};

template <typename T, int KMAX>
__global__ __launch_bounds__(kThreads) void k_update(int n, int j, T* __restrict__ W,
                                                     const State* __restrict__ st, size_t bs) {
  typedef typename Vec16<T>::type V;
  constexpr int kV = (int)(16 / sizeof(T));
  st = bat(st, bs);
  if (st->brk || st->done) return;
  W = bat(W, bs);
  const int lo = st->step_lo, nw = j - lo + 1;
  // FP64 arithmetic for either value type: z is nearly in the span of the window, so the
  // difference cancels; only the stored w_{j+1} is rounded to T.
  const double inv = st->inv_rho;
  double coef[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) coef[q] = (q < nw) ? st->upd_coef[q] : 0.0;
  const size_t ld = wcol(n, sizeof(T));
  T* out = W + (size_t)(j + 1) * ld;
  const T* base = W + (size_t)lo * ld;
  const int nv = n / kV;
  const int stride = (int)gridDim.x * kThreads;
  const int t0 = (int)blockIdx.x * kThreads + (int)threadIdx.x;
  for (int i = t0; i < nv; i += stride) {
    const V zv = __builtin_nontemporal_load(reinterpret_cast<const V*>(out) + i);
    V wv[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < nw) wv[q] = __builtin_nontemporal_load(reinterpret_cast<const V*>(base + (size_t)q * ld) + i);
    V r;
#pragma unroll
    for (int e = 0; e < kV; ++e) {
      double v = (double)zv[e];
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (q < nw) v -= coef[q] * (double)wv[q][e];
      r[e] = (T)(v * inv);
    }
    __builtin_nontemporal_store(r, reinterpret_cast<V*>(out) + i);
  }
  for (int i = nv * kV + t0; i < n; i += stride) {  // the last n mod kV elements
    double v = (double)out[i];
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < nw) v -= coef[q] * (double)base[(size_t)q * ld + i];
    out[i] = (T)(v * inv);
  }
}

// The same update for wide windows (k > 8, up to the whole basis: the k = m update of the paper's
// restart-rand and unrestarted rand, a tall-skinny product, Section 2.2).  The coefficients come
// from LDS instead of registers (64 FP64 coefficients per thread cost the occupancy), the columns
// in groups of kUpdGroup whose loads are issued together, two adjacent rows per thread (16-byte
// loads for FP64).  The arithmetic and its order are k_update's, so the bits are the same.
constexpr int kUpdGroup = 8;

template <typename T>
struct Pair;
template <>
struct Pair<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};

template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_wide(int n, int j, T* __restrict__ W,
                                                          const State* __restrict__ st, size_t bs) {
  typedef typename Pair<T>::type P;
  __shared__ double s_coef[kMaxM + 1];
  st = bat(st, bs);
  if (st->brk || st->done) return;
  W = bat(W, bs);
  const int lo = st->step_lo, nw = j - lo + 1;
  for (int q = threadIdx.x; q < nw; q += kThreads) s_coef[q] = st->upd_coef[q];
  const double inv = st->inv_rho;
  __syncthreads();
  const size_t ld = wcol(n, sizeof(T));  // whole 4 KiB pages: every column's pairs are aligned
  T* out = W + (size_t)(j + 1) * ld;
  const T* base = W + (size_t)lo * ld;
  const size_t npair = ((size_t)n + 1) / 2;
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t pi = (size_t)blockIdx.x * kThreads + threadIdx.x; pi < npair; pi += stride) {
    const size_t i = 2 * pi;
    const bool two = i + 1 < (size_t)n;
    double v0, v1 = 0.0;
    if (two) {
      const P zz = __builtin_nontemporal_load(reinterpret_cast<const P*>(out + i));
      v0 = (double)zz.x;
      v1 = (double)zz.y;
    } else {
      v0 = (double)__builtin_nontemporal_load(out + i);
    }
    for (int q0 = 0; q0 < nw; q0 += kUpdGroup) {
      P a[kUpdGroup];
#pragma unroll
      for (int u = 0; u < kUpdGroup; ++u) {
        const int q = q0 + u;
        a[u] = P{T(0), T(0)};
        if (q < nw) {
          const T* col = base + (size_t)q * ld + i;
          if (two) a[u] = __builtin_nontemporal_load(reinterpret_cast<const P*>(col));
          else a[u].x = __builtin_nontemporal_load(col);
        }
      }
#pragma unroll
      for (int u = 0; u < kUpdGroup; ++u) {
        if (q0 + u < nw) {
          const double c = s_coef[q0 + u];
          v0 -= c * (double)a[u].x;
          v1 -= c * (double)a[u].y;
        }
      }
    }
    if (two) {
      P r;
      r.x = (T)(v0 * inv);
      r.y = (T)(v1 * inv);
      __builtin_nontemporal_store(r, reinterpret_cast<P*>(out + i));
    } else {
      __builtin_nontemporal_store((T)(v0 * inv), out + i);
    }
  }
}

// ------------------------------------------------------------------ plain Arnoldi (CGS2) kernels
// Partial Gram products h_i = <V_i, z>, i < j1, plus ||z||^2 in slot entry j1 when want_norm.
// Columns in chunks of kGramCols (one pass over the rows per chunk, z read again for each).
constexpr int kGramCols = 8;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram(int n, int j1, const T* __restrict__ V,
                                                   const T* __restrict__ z, double* __restrict__ slots,
                                                   int want_norm, const State* __restrict__ st) {
  __shared__ double part[kThreads / 64][kMaxM + 2];
  if (st->brk) return;
  const int ncol = j1 + (want_norm ? 1 : 0);
  typedef typename Pair<T>::type P;
  const size_t ld = wcol(n, sizeof(T));  // whole 4 KiB pages: every column's pairs are aligned
  const size_t npair = ((size_t)n + 1) / 2;
  const size_t stride = (size_t)gridDim.x * kThreads;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c0 = 0; c0 < ncol; c0 += kGramCols) {
    double acc[kGramCols];
#pragma unroll
    for (int q = 0; q < kGramCols; ++q) acc[q] = 0.0;
    // two adjacent rows per thread (16-byte loads for FP64)
    for (size_t pi = (size_t)blockIdx.x * kThreads + threadIdx.x; pi < npair; pi += stride) {
      const size_t i = 2 * pi;
      const bool two = i + 1 < (size_t)n;
      P zz = P{T(0), T(0)};
      if (two) zz = *reinterpret_cast<const P*>(z + i);
      else zz.x = z[i];
      const double z0 = (double)zz.x, z1 = (double)zz.y;
#pragma unroll
      for (int q = 0; q < kGramCols; ++q) {
        const int c = c0 + q;
        if (c < j1) {
          P a = P{T(0), T(0)};
          if (two) a = *reinterpret_cast<const P*>(V + (size_t)c * ld + i);
          else a.x = V[(size_t)c * ld + i];
          acc[q] += (double)a.x * z0 + (double)a.y * z1;
        } else if (c == j1 && want_norm) {
          acc[q] += z0 * z0 + z1 * z1;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kGramCols; ++q) {
      const double s = wave_sum(acc[q]);
      if (lane == 0 && c0 + q < ncol) part[w][c0 + q] = s;
    }
  }
  __syncthreads();
  double* slot = slots + (size_t)(blockIdx.x % kSlots) * (kMaxM + 2);
  for (int c = threadIdx.x; c < ncol; c += kThreads) {
    double s = 0.0;
    for (int q = 0; q < (kThreads / 64); ++q) s += part[q][c];
    unsafeAtomicAdd(slot + c, s);
  }
}

// z -= V h with h = sum of the slot copies; accumulates ||z||^2 into norm slots when want_norm.
// Block 0 adds h into the Hessenberg column j and zeroes `slots_zero` (the other pass's set).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cgs_update(int n, int j, int m, T* __restrict__ V,
                                                         const double* __restrict__ slots,
                                                         double* __restrict__ slots_zero,
                                                         double* __restrict__ norm_slots, int want_norm,
                                                         double* __restrict__ R, State* __restrict__ st) {
  __shared__ double h[kMaxM + 1];
  __shared__ double red[2 * (kThreads / 64)];
  int phase = 0;
  if (st->brk) return;
  const int j1 = j + 1;
  for (int c = threadIdx.x; c < j1; c += kThreads) {
    double s = 0.0;
    for (int q = 0; q < kSlots; ++q) s += slots[(size_t)q * (kMaxM + 2) + c];
    h[c] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int c = threadIdx.x; c < j1; c += kThreads) R[(size_t)j * (m + 1) + c] += h[c];
    if (!want_norm && threadIdx.x == 0) {  // pass 1 carries ||z||^2 before orthogonalization
      double r2 = 0.0;
      for (int q = 0; q < kSlots; ++q) r2 += slots[(size_t)q * (kMaxM + 2) + j1];
      st->raw2 = r2;
    }
    for (int c = threadIdx.x; c < kSlots * (kMaxM + 2); c += kThreads) slots_zero[c] = 0.0;
  }
  // two adjacent rows per thread, the basis columns in groups of kUpdGroup whose loads are issued
  // together (one load in flight per column otherwise); column order as before
  typedef typename Pair<T>::type P;
  const size_t ld = wcol(n, sizeof(T));  // whole 4 KiB pages: every column's pairs are aligned
  T* z = V + (size_t)j1 * ld;
  const size_t npair = ((size_t)n + 1) / 2;
  const size_t stride = (size_t)gridDim.x * kThreads;
  double nrm = 0.0;
  for (size_t pi = (size_t)blockIdx.x * kThreads + threadIdx.x; pi < npair; pi += stride) {
    const size_t i = 2 * pi;
    const bool two = i + 1 < (size_t)n;
    double v0, v1 = 0.0;
    if (two) {
      const P zz = *reinterpret_cast<const P*>(z + i);
      v0 = (double)zz.x;
      v1 = (double)zz.y;
    } else {
      v0 = (double)z[i];
    }
    for (int c0 = 0; c0 < j1; c0 += kUpdGroup) {
      P a[kUpdGroup];
#pragma unroll
      for (int u = 0; u < kUpdGroup; ++u) {
        a[u] = P{T(0), T(0)};
        if (c0 + u < j1) {
          const T* col = V + (size_t)(c0 + u) * ld + i;
          if (two) a[u] = *reinterpret_cast<const P*>(col);
          else a[u].x = *col;
        }
      }
#pragma unroll
      for (int u = 0; u < kUpdGroup; ++u) {
        if (c0 + u < j1) {
          v0 -= h[c0 + u] * (double)a[u].x;
          v1 -= h[c0 + u] * (double)a[u].y;
        }
      }
    }
    const T t0 = (T)v0, t1 = (T)v1;
    if (two) {
      P r;
      r.x = t0;
      r.y = t1;
      *reinterpret_cast<P*>(z + i) = r;
    } else {
      z[i] = t0;
    }
    nrm += (double)t0 * (double)t0 + (double)t1 * (double)t1;
  }
  if (want_norm) {
    const double s = block_sum(nrm, red, phase);
    if (threadIdx.x == 0) unsafeAtomicAdd(norm_slots + (blockIdx.x % kSlots), s);
  }
}

// rho = ||z|| after CGS2; Hessenberg entry, breakdown test against the raw norm kept by pass 1.
__global__ void k_plain_finish(int j, int m, double* __restrict__ norm_slots, double* __restrict__ R,
                               State* __restrict__ st) {
  if (threadIdx.x != 0 || st->brk) return;
  double s = 0.0;
  for (int q = 0; q < kSlots; ++q) {
    s += norm_slots[q];
    norm_slots[q] = 0.0;
  }
  const double raw = st->raw2;
  const double rho = sqrt(s);
  const bool finite = isfinite(rho) && isfinite(raw);
  if (!finite || !(rho > 64.0 * 2.220446049250313e-16 * sqrt(raw))) {
    st->brk = 1;
    st->meff = j + 1;
    if (!finite) st->nonfinite = 1;
    return;
  }
  R[(size_t)j * (m + 1) + j + 1] = rho;
  st->inv_rho = 1.0 / rho;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale_col(int n, T* __restrict__ v, const double* __restrict__ s_ptr,
                                                        const State* __restrict__ st, size_t bs) {
  st = bat(st, bs);
  if (st->brk || st->done) return;
  v = bat(v, bs);
  s_ptr = bat(s_ptr, bs);
  const T s = (T)(*s_ptr);
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < (size_t)n; i += stride) v[i] *= s;
}

// ------------------------------------------------------------------------------------ launchers
static int zeta_bucket(int zeta) { return zeta <= 1 ? 1 : zeta <= 4 ? 4 : zeta <= 8 ? 8 : zeta <= 16 ? 16 : 32; }

size_t spmv_sketch_lds(int dtype, int mode, int d, int G, int zeta, bool c16) {
  const size_t es = dtype == 0 ? 8 : 4;
  const size_t chunk = (mode == 1) ? 0 : (size_t)kChunk * (es + (c16 && G <= 1 ? 2 : 4));
  if (G > 1) return grp_lds_bins(d, G) + grp_lds_table(zeta_bucket(zeta)) + chunk;
  return spmv_lds_bins(mode, d) + chunk;
}

// A launch that, when timing events are given, has the dispatch itself record them at the kernel's
// start and end (hipExtLaunchKernelGGL): the interval is the kernel's own, as in a trace, without
// the gap a separate event record leaves before the dispatch.
template <typename K, typename... Args>
static void launch_timed(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, e0, e1, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

template <typename T>
static hipError_t launch_spmv_sketch_t(hipStream_t s, int mode, int grid, int n, const int* rp, const int* ci,
                                       const int16_t* cr, const T* va, const T* x, T* y, int d, int zeta, uint64_t seed,
                                       double* parts, const State* st, int nb, int G, size_t bs, int nts,
                                       hipEvent_t e0, hipEvent_t e1) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const T scale = (T)(1.0 / sqrt((double)zeta));
  if (G > 1 && (mode == 2 || G % kWaves != 0 || G > kGroupMax || (int64_t)n * (int64_t)sizeof(T) > INT32_MAX))
    return hipErrorInvalidValue;
  const size_t lds = spmv_sketch_lds(sizeof(T) == 8 ? 0 : 1, mode, d, G, zeta, cr != nullptr);
  const dim3 g2(grid, (nb + G - 1) / G);
  const bool c16 = cr != nullptr && mode != 1;  // the sketch-only mode stages no CSR chunk
#define FAB_L(M, Z)                                                                                                \
  if (G > 1)                                                                                                       \
    launch_timed(k_spmv_sketch_grp<T, M, Z>, g2, dim3(kThreads), lds, s, e0, e1, n, rp, ci, cr, va, x, y, d, zeta,   \
                 scale, k0, k1, parts, st, nb, G, bs);                                                             \
  else if (c16)                                                                                                    \
    launch_timed(k_spmv_sketch<T, M, Z, (M != 1)>, g2, dim3(kThreads), lds, s, e0, e1, n, rp, ci, cr, va, x, y, d,   \
                 zeta, scale, k0, k1, parts, st, bs, nts);                                                         \
  else                                                                                                             \
    launch_timed(k_spmv_sketch<T, M, Z>, g2, dim3(kThreads), lds, s, e0, e1, n, rp, ci, cr, va, x, y, d, zeta,       \
                 scale, k0, k1, parts, st, bs, nts)
#define FAB_LS(Z)                                                                                                  \
  if (c16)                                                                                                         \
    launch_timed(k_spmv_sketch<T, 2, Z, true>, g2, dim3(kThreads), lds, s, e0, e1, n, rp, ci, cr, va, x, y, d, zeta, \
                 scale, k0, k1, parts, st, bs, nts);                                                               \
  else                                                                                                             \
    launch_timed(k_spmv_sketch<T, 2, Z>, g2, dim3(kThreads), lds, s, e0, e1, n, rp, ci, cr, va, x, y, d, zeta,       \
                 scale, k0, k1, parts, st, bs, nts)
#define FAB_Z(M)           \
  if (zeta <= 1) {         \
    FAB_L(M, 1);           \
  } else if (zeta <= 4) {  \
    FAB_L(M, 4);           \
  } else if (zeta <= 8) {  \
    FAB_L(M, 8);           \
  } else if (zeta <= 16) { \
    FAB_L(M, 16);          \
  } else {                 \
    FAB_L(M, 32);          \
  }
  if (mode == 0) {
    FAB_Z(0)
  } else if (mode == 1) {
    FAB_Z(1)
  } else {
    FAB_LS(1);
  }
#undef FAB_Z
#undef FAB_LS
#undef FAB_L
  return hipGetLastError();
}

constexpr int kGroupLdsMax = 96 * 1024;   // dynamic LDS the grouped kernel may use
constexpr int kSpmvLdsMax = 160 * 1024;   // one member per block: up to the whole LDS of a CU (d up to
                                          // kMaxD: four wavefront bin sets of 32 KB and the CSR chunk)

template <typename T, int M, int Z>
static hipError_t configure_mz() {
  hipError_t e = hipSuccess;
  if (M != 2)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spmv_sketch_grp<T, (M == 2 ? 0 : M), Z>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kGroupLdsMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spmv_sketch<T, M, Z>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kSpmvLdsMax);
  if (e == hipSuccess && M != 1)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spmv_sketch<T, M, Z, (M != 1)>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kSpmvLdsMax);
  return e;
}

template <typename T>
static hipError_t configure_t() {
  hipError_t e = hipSuccess;
  const hipError_t es[] = {configure_mz<T, 0, 1>(), configure_mz<T, 0, 4>(), configure_mz<T, 0, 8>(),
                           configure_mz<T, 0, 16>(), configure_mz<T, 0, 32>(), configure_mz<T, 1, 1>(),
                           configure_mz<T, 1, 4>(), configure_mz<T, 1, 8>(), configure_mz<T, 1, 16>(),
                           configure_mz<T, 1, 32>(), configure_mz<T, 2, 1>()};
  for (hipError_t x : es)
    if (x != hipSuccess) e = x;
  return e;
}

// Dynamic LDS limits of the fused kernel's instantiations (beyond the default 64 KB).
hipError_t configure_step_kernels() {
  const hipError_t e = configure_t<double>();
  return e != hipSuccess ? e : configure_t<float>();
}

size_t group_lds_max() { return kGroupLdsMax; }

// The instantiation launch_spmv_sketch picks, for the occupancy query below.
template <typename T, int M, int Z>
static const void* spmv_kernel_mz(int G, bool c16) {
  if (G > 1 && M != 2) return reinterpret_cast<const void*>(&k_spmv_sketch_grp<T, (M == 2 ? 0 : M), Z>);
  if (c16 && M != 1) return reinterpret_cast<const void*>(&k_spmv_sketch<T, M, Z, (M != 1)>);
  return reinterpret_cast<const void*>(&k_spmv_sketch<T, M, Z>);
}

template <typename T>
static const void* spmv_kernel(int mode, int zeta, int G, bool c16) {
  if (mode == 2) return spmv_kernel_mz<T, 2, 1>(G, c16);
  const int Z = zeta_bucket(zeta);
  if (mode == 0) {
    switch (Z) {
      case 1: return spmv_kernel_mz<T, 0, 1>(G, c16);
      case 4: return spmv_kernel_mz<T, 0, 4>(G, c16);
      case 8: return spmv_kernel_mz<T, 0, 8>(G, c16);
      case 16: return spmv_kernel_mz<T, 0, 16>(G, c16);
      default: return spmv_kernel_mz<T, 0, 32>(G, c16);
    }
  }
  switch (Z) {
    case 1: return spmv_kernel_mz<T, 1, 1>(G, c16);
    case 4: return spmv_kernel_mz<T, 1, 4>(G, c16);
    case 8: return spmv_kernel_mz<T, 1, 8>(G, c16);
    case 16: return spmv_kernel_mz<T, 1, 16>(G, c16);
    default: return spmv_kernel_mz<T, 1, 32>(G, c16);
  }
}

// Blocks of the fused kernel resident per CU, from the runtime's occupancy calculator (registers,
// LDS with its allocation granularity, wavefront slots), so that a grid of that many blocks per CU
// runs in one pass with no trailing partial wave of blocks.
int spmv_blocks_per_cu(int dtype, int mode, int d, int G, int zeta, bool c16) {
  const size_t lds = spmv_sketch_lds(dtype, mode, d, G, zeta, c16);
  const void* f = dtype == 0 ? spmv_kernel<double>(mode, zeta, G, c16) : spmv_kernel<float>(mode, zeta, G, c16);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kThreads, lds) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

hipError_t launch_spmv_sketch(hipStream_t s, int dtype, int mode, int grid, int n, const int* rp, const int* ci,
                              const int16_t* cr, const void* va, const void* x, void* y, int d, int zeta, uint64_t seed,
                              double* parts, const State* st, int nb, int G, size_t bs, int nts, hipEvent_t e0,
                              hipEvent_t e1) {
  // the partials need a grid of whole XCD rounds within the partial buffer (part_index)
  if (mode != 2 && (grid < kXcds || grid > kMaxParts || grid % kXcds != 0)) return hipErrorInvalidValue;
  if (dtype == 0)
    return launch_spmv_sketch_t<double>(s, mode, grid, n, rp, ci, cr, (const double*)va, (const double*)x,
                                        (double*)y, d, zeta, seed, parts, st, nb, G, bs, nts, e0, e1);
  return launch_spmv_sketch_t<float>(s, mode, grid, n, rp, ci, cr, (const float*)va, (const float*)x, (float*)y, d,
                                     zeta, seed, parts, st, nb, G, bs, nts, e0, e1);
}

hipError_t launch_reduce_parts(hipStream_t s, int e0, int len, int nparts, const double* parts, double* out,
                               const State* st, int skip, int nb, size_t bs) {
  if (len < 1) return hipSuccess;
  if (nparts < 1 || nparts > kMaxParts) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_parts, dim3(len, nb), dim3(kThreads), 0, s, e0, nparts, parts, out, st, skip, bs);
  return hipGetLastError();
}

hipError_t launch_orth(hipStream_t s, int j, int k, int m, int d, const double* uraw, double* U, double* R,
                       State* st, int nb, size_t bs) {
  const dim3 g(1, nb);
  if (d <= 256)
    hipLaunchKernelGGL(k_orth<4>, g, dim3(64), 0, s, j, k, m, d, uraw, U, R, st, bs);
  else if (d <= 512)
    hipLaunchKernelGGL(k_orth<8>, g, dim3(64), 0, s, j, k, m, d, uraw, U, R, st, bs);
  else if (d <= 1024)
    hipLaunchKernelGGL(k_orth<16>, g, dim3(64), 0, s, j, k, m, d, uraw, U, R, st, bs);
  else if (d <= 2048)
    hipLaunchKernelGGL(k_orth<32>, g, dim3(64), 0, s, j, k, m, d, uraw, U, R, st, bs);
  else
    hipLaunchKernelGGL(k_orth<64>, g, dim3(64), 0, s, j, k, m, d, uraw, U, R, st, bs);
  return hipGetLastError();
}

hipError_t launch_orth_update(hipStream_t s, int dtype, int num_cu, int n, int j, int k, int m, int d, void* W,
                              const double* uraw, double* U, double* R, double* G, State* st, int nb, size_t bs,
                              const double* parts, int nparts, int nts, hipEvent_t e0, hipEvent_t e1) {
  if (parts && (nparts < 1 || nparts > 64)) return hipErrorInvalidValue;  // one partial per lane
  const int ob = dtype == 0 ? (nts ? OuBatch<double, kAuxNt>::v : OuBatch<double, 0>::v)
                            : (nts ? OuBatch<float, kAuxNt>::v : OuBatch<float, 0>::v);
  const int nbat = (int)((n + ob - 1) / ob);
  const int grid = std::max(1, std::min(nbat, ou_blocks_per_cu(nts) * num_cu));
  const dim3 g(grid, nb);
#define FAB_OU2(TT, KK, INL, AUX)                                                                              \
  launch_timed(k_orth_update<TT, KK, INL, AUX>, g, dim3(kOuThreads), 0, s, e0, e1, n, j, k, m, d, (TT*)W, uraw, U, R, \
               G, st, bs, parts, nparts)
#define FAB_OU(TT, KK)               \
  if (parts) {                       \
    if (nts) {                       \
      FAB_OU2(TT, KK, true, kAuxNt); \
    } else {                         \
      FAB_OU2(TT, KK, true, 0);      \
    }                                \
  } else if (nts) {                  \
    FAB_OU2(TT, KK, false, kAuxNt);  \
  } else {                           \
    FAB_OU2(TT, KK, false, 0);       \
  }
  if (dtype == 0) {
    if (k <= 4) {
      FAB_OU(double, 4)
    } else {
      FAB_OU(double, 8)
    }
  } else {
    if (k <= 4) {
      FAB_OU(float, 4)
    } else {
      FAB_OU(float, 8)
    }
  }
#undef FAB_OU
#undef FAB_OU2
  return hipGetLastError();
}

template <typename T>
static void launch_update_t(hipStream_t s, int grid, int n, int j, int k, T* W, const State* st, int nb, size_t bs,
                            hipEvent_t e0, hipEvent_t e1) {
  const dim3 g(grid, nb);
  // k_update: one 16-byte vector per thread and trip, so a quarter (FP32) or half (FP64) of the
  // element grid, in whole XCD rounds
  const int nv = n / (int)(16 / sizeof(T));
  const int gv = std::max(kXcds, std::min(grid, ((nv + kThreads - 1) / kThreads + kXcds - 1) / kXcds * kXcds));
  const dim3 g16(gv, nb);
  if (k <= 4)
    launch_timed(k_update<T, 4>, g16, dim3(kThreads), 0, s, e0, e1, n, j, W, st, bs);
  else if (k <= 8)
    launch_timed(k_update<T, 8>, g16, dim3(kThreads), 0, s, e0, e1, n, j, W, st, bs);
  else
    launch_timed(k_update_wide<T>, g, dim3(kThreads), 0, s, e0, e1, n, j, W, st, bs);
}

hipError_t launch_update(hipStream_t s, int dtype, int grid, int n, int j, int k, void* W, const State* st, int nb,
                         size_t bs, hipEvent_t e0, hipEvent_t e1) {
  if (dtype == 0)
    launch_update_t<double>(s, grid, n, j, k, (double*)W, st, nb, bs, e0, e1);
  else
    launch_update_t<float>(s, grid, n, j, k, (float*)W, st, nb, bs, e0, e1);
  return hipGetLastError();
}

hipError_t launch_gram(hipStream_t s, int dtype, int grid, int n, int j1, const void* V, const void* z,
                       double* slots, int want_norm, const State* st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_gram<double>, dim3(grid), dim3(kThreads), 0, s, n, j1, (const double*)V,
                       (const double*)z, slots, want_norm, st);
  else
    hipLaunchKernelGGL(k_gram<float>, dim3(grid), dim3(kThreads), 0, s, n, j1, (const float*)V,
                       (const float*)z, slots, want_norm, st);
  return hipGetLastError();
}

hipError_t launch_cgs_update(hipStream_t s, int dtype, int grid, int n, int j, int m, void* V, const double* slots,
                             double* slots_zero, double* norm_slots, int want_norm, double* R, State* st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_cgs_update<double>, dim3(grid), dim3(kThreads), 0, s, n, j, m, (double*)V, slots,
                       slots_zero, norm_slots, want_norm, R, st);
  else
    hipLaunchKernelGGL(k_cgs_update<float>, dim3(grid), dim3(kThreads), 0, s, n, j, m, (float*)V, slots,
                       slots_zero, norm_slots, want_norm, R, st);
  return hipGetLastError();
}

hipError_t launch_plain_finish(hipStream_t s, int j, int m, double* norm_slots, double* R, State* st) {
  hipLaunchKernelGGL(k_plain_finish, dim3(1), dim3(64), 0, s, j, m, norm_slots, R, st);
  return hipGetLastError();
}

hipError_t launch_scale_col(hipStream_t s, int dtype, int grid, int n, void* v, const double* s_ptr,
                            const State* st, int nb, size_t bs) {
  const dim3 g(grid, nb);
  if (dtype == 0)
    hipLaunchKernelGGL(k_scale_col<double>, g, dim3(kThreads), 0, s, n, (double*)v, s_ptr, st, bs);
  else
    hipLaunchKernelGGL(k_scale_col<float>, g, dim3(kThreads), 0, s, n, (float*)v, s_ptr, st, bs);
  return hipGetLastError();
}

}  // namespace fab
