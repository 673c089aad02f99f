// Dense n_u x n_u stages: the global sum of the scenario contributions (the
// paper's MPI all-reduce of K_hat, here a fixed-order on-device sum), the
// Cholesky factorisation of K_hat (the paper factorises it densely with
// LAPACK on the GPU) and the two triangular solves for p_u.
#include <utility>

#include "device.h"

namespace rkkt {

namespace {

constexpr int kThreads = 256;
constexpr int kNB = 64;          // panel width of the blocked factorisation
constexpr int kSmallN = 128;     // whole matrix (padded to a multiple of 16) in LDS up to this order
constexpr int kWavesD = kThreads / 64;

__global__ void k_set_int(int* p, int v) { *p = v; }

// K_hat = sum_c src_c + diag(sigma_u) + delta_w I over `cnt` n_u x n_u
// matrices (the scenario contributions, or the chunk partials of the stacked
// product), lower triangle, mirrored into the upper one so K_hat is exactly
// symmetric.  A workgroup of kE * kW threads owns kE entries of the lower
// triangle (row-major order); its kW groups of kE threads each sum a
// contiguous share of the matrices in index order, and the kW partial sums
// are added in a fixed order (in groups of eight first when kW > 16), so the
// result does not depend on scheduling.  Few matrices (the scenario
// contributions): 64 entries x 16 groups; many (the 256 chunk partials): 16
// entries x 64 groups, so that four times as many workgroups share the reads.
constexpr int kSumEntries = 64, kSumWaves = 16;
constexpr int kSumEntriesMany = 16, kSumWavesMany = 64;
constexpr int kSumManyFrom = 128;  // matrices from which the second shape is used

template <int kE, int kW>
__device__ __forceinline__ void sym_sum_body(int bx_, const DP& d, const double* src, int cnt, const double* su,
                                             double dw, double* khat) {
  static_assert(kW <= 16 || kW % 8 == 0, "partials in groups of eight");
  constexpr int kG = kW > 16 ? kW / 8 : kW;  // partials left after the grouping
  __shared__ double part[kW][kE];
  __shared__ double part2[kW > 16 ? kG : 1][kE];
  const int n = d.nu;
  const long long nn = (long long)n * n, ntri = (long long)n * (n + 1) / 2;
  const int lane = threadIdx.x % kE, wv = threadIdx.x / kE;
  const long long t = (long long)bx_ * kE + lane;
  // t -> (r, c), c <= r, rows in order
  int r = 0, c = 0;
  if (t < ntri) {
    r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long long)r * (r + 1) / 2 > t) --r;
    while ((long long)(r + 1) * (r + 2) / 2 <= t) ++r;
    c = (int)(t - (long long)r * (r + 1) / 2);
  }
  const long long off = (long long)r * n + c;
  const int per = (cnt + kW - 1) / kW;
  const int k0 = wv * per, k1 = min(cnt, k0 + per);
  double acc = 0.0;
  if (t < ntri) {
    // loads in batches of 16 so that they are in flight together; the
    // additions keep the matrix order
    for (int k = k0; k < k1; k += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = k + u < k1 ? src[(long long)(k + u) * nn + off] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (k + u < k1) acc += v[u];
    }
  }
  part[wv][lane] = acc;
  __syncthreads();
  const double* fin = &part[0][0];
  if constexpr (kW > 16) {
    if (wv < kG) {
      double s2 = part[8 * wv][lane];
#pragma unroll
      for (int q = 1; q < 8; ++q) s2 += part[8 * wv + q][lane];
      part2[wv][lane] = s2;
    }
    __syncthreads();
    fin = &part2[0][0];
  }
  if (wv == 0 && t < ntri) {
    double s = fin[lane];
    for (int q = 1; q < kG; ++q) s += fin[q * kE + lane];
    if (r == c) s += su[r] + dw;
    if (!isfinite(s)) atomicCAS(d.status, 0, RKKT_ERR_NONFINITE);
    khat[off] = s;
    khat[(long long)c * n + r] = s;
  }
}

template <int kE, int kW>
__global__ __launch_bounds__(kE * kW) void k_sym_sum(DP d, const double* src, int cnt, const double* su, double dw,
                                                     double* khat) {
  sym_sum_body<kE, kW>((int)blockIdx.x, d, src, cnt, su, dw, khat);
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Stacked product of the reduction's product variant: for chunk c of the
// stacked rows rho (all scenarios, x rows then u rows of each),
//   gpart_c[i][j] = sum_rho Z[rho][i] (K Z)[rho][j],   i >= j,
// so that sum_c gpart_c = sum_k Z_k^T K_k Z_k.  The output's lower triangle
// is cut into 16 x 16 blocks, grouped into super-tiles of kSB x kSB blocks
// (triangular on the diagonal).  One workgroup per (super-tile, chunk): it
// streams the chunk's rows in slabs of kSpSlab rows (the super-tile's 16 kSB
// columns of Z and of K Z) straight from global memory into LDS
// (global_load_lds_dwordx4, no registers held), four slab buffers deep with
// three slabs in flight, and its 4 wavefronts take the super-tile's blocks
// round robin, each block one v_mfma_f64_16x16x4f64 accumulator (A operand:
// lane holds Z[rho + lane/16][i + lane%16]; B operand: (K Z)[rho +
// lane/16][j + lane%16]; result register r of a lane: row lane/16 + 4 r,
// column lane%16).  Chunks are whole slabs except the last, whose rows past
// the last stacked row are zero rows of the panels, so they add nothing.
constexpr int kSB = 7;                        // blocks per super-tile side
constexpr int kSBMax = (kSB * kSB + 3) / 4;   // blocks per wavefront, at most
constexpr int kSpCols = 16 * kSB;             // columns of a slab part (Z or K Z), LDS row pitch
constexpr int kSpPart = kSpSlab * kSpCols;    // doubles of one part of a slab
constexpr int kSpLoads = 2 * kSpPart / 128;   // 1 KiB wavefront loads per slab (64 lanes x 16 bytes)
constexpr int kSpPerWave = kSpLoads / 4;
static_assert(kSpPart % 128 == 0 && kSpLoads % 4 == 0, "slab loads: whole 1 KiB units, four wavefronts");
static_assert(kSpCols % 2 == 0, "a lane's two doubles stay in one row");

__host__ __device__ inline int sp_nblk(int nu) { return (nu + 15) / 16; }
__host__ __device__ inline int sp_nsuper(int nu) { return (sp_nblk(nu) + kSB - 1) / kSB; }
__host__ __device__ inline long long sp_rows_per_chunk(long long rows, int nchunk) {
  return ((rows + nchunk - 1) / nchunk + kSpSlab - 1) / kSpSlab * kSpSlab;
}

__shared__ double sp_buf0[2 * kSpPart], sp_buf1[2 * kSpPart], sp_buf2[2 * kSpPart], sp_buf3[2 * kSpPart];

// s_waitcnt immediates (vmcnt in bits 3:0, expcnt and lgkmcnt at their
// maxima): all but the loads of the last two slabs, or all
constexpr int kWaitVm2Slabs = 0x0F70 | (2 * kSpPerWave);
constexpr int kWaitVm0 = 0x0F70;
static_assert(2 * kSpPerWave < 16, "vmcnt wait fits the low field");

// workgroup barrier that the compiler may not move memory accesses across;
// the hardware waits are explicit (the slab loads in flight must stay so)
__device__ __forceinline__ void sp_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// kSlots: blocks per wavefront for this shape; every slot's product runs
// (a slot past the wavefront's blocks reads block (0, 0) and is not stored),
// so the accumulators stay in fixed registers with no branches around them
template <int kSlots>
__device__ __forceinline__ void stacked_product_body(int bx_, int by_, int gx_, const DP& d, long long per) {
  int t = bx_, SI = 0;
  while (t > SI) { t -= SI + 1; ++SI; }
  const int SJ = t, chunk = by_;
  const int nblk = sp_nblk(d.nu);
  const int bi0 = SI * kSB, bj0 = SJ * kSB;
  const int ni = min(kSB, nblk - bi0), nj = min(kSB, nblk - bj0);
  const long long rows = (long long)d.N * d.nz;
  const long long r0 = (long long)chunk * per, r1 = min(rows, r0 + per);
  const int nsl = r1 > r0 ? (int)((r1 - r0 + kSpSlab - 1) / kSpSlab) : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lm = lane & 15, lk = lane >> 4;
  const long long ld = d.nu_pad;
  // this wavefront's blocks: numbers wv, wv + 4, ... of the super-tile's
  // blocks (a, b) in row order (lower triangle on the diagonal), a over Z,
  // b over K Z
  const int nblocks = SI == SJ ? ni * (ni + 1) / 2 : ni * nj;
  int ba[kSlots], bb[kSlots];
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    int idx = wv + 4 * q, a = 0;
    if (idx >= nblocks) {
      idx = 0;
    } else if (SI == SJ) {
      while (idx > a) { idx -= a + 1; ++a; }
    } else {
      a = idx / nj;
      idx -= a * nj;
    }
    ba[q] = a;
    bb[q] = idx;
  }
  const int nmine = nblocks > wv ? (nblocks - wv + 3) / 4 : 0;
  v4d acc[kSlots];
#pragma unroll
  for (int q = 0; q < kSlots; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  // slab loads: load u of this wavefront moves 128 doubles of one part (Z
  // for the first kSpLoads / 2 loads of the slab, K Z after) to LDS offset
  // 128 g of that part, g its number within the part; lane l brings the
  // two doubles at (row, col) = divmod(128 g + 2 l, kSpCols).  Columns past
  // the super-tile's blocks repeat its last two columns (in bounds; no
  // stored block reads them).
  // Slab loads go through buffer resources whose base is the chunk's first
  // row (of the super-tile's columns): the lane offsets (bytes from a slab's
  // first row) stay fixed in their registers and the slab's offset is a
  // scalar operand, so no register read by a load in flight is rewritten.
  // Load u of this wavefront moves 128 doubles of one part (Z for the first
  // kSpLoads / 2 loads of the slab, K Z after) to LDS offset 128 g of that
  // part, g its number within the part; lane l brings the two doubles at
  // (row, col) = divmod(128 g + 2 l, kSpCols).  Columns past the
  // super-tile's blocks repeat its last two columns (no stored block reads
  // them).
  const long long pbytes = ((long long)rows + kSpSlab) * ld * 8;  // panel allocation
  auto rsrc = [&](const double* panel, int colblk) {
    const long long off = (r0 * ld + 16LL * colblk) * 8;
    const long long left = pbytes - off;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(reinterpret_cast<const char*>(panel) + off),
                                             (short)0, (int)min(left, 0x7fffffffLL), 0x00020000);
  };
  const __amdgpu_buffer_rsrc_t rz = rsrc(d.Zst, bi0), rk = rsrc(d.KZst, bj0);
  // a resource with no records: loads through it return zeros without
  // touching memory (the slabs past the chunk's last one, which keep the
  // pipeline's wait counts uniform and are never multiplied)
  const __amdgpu_buffer_rsrc_t rnone = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(d.Zst), (short)0, 0, 0x00020000);
  int voff[kSpPerWave], loff[kSpPerWave];
  bool pk[kSpPerWave];
#pragma unroll
  for (int u = 0; u < kSpPerWave; ++u) {
    const int ti = wv * kSpPerWave + u, part = ti >= kSpLoads / 2, g = part ? ti - kSpLoads / 2 : ti;
    const int e = 128 * g + 2 * lane, row = e / kSpCols, col = e % kSpCols;
    const int lim = 16 * (part ? nj : ni);
    pk[u] = part;
    voff[u] = 8 * (row * (int)ld + min(col, lim - 2));
    loff[u] = part * kSpPart + 128 * g;
  }
  auto issue = [&](double* buf, int s) {
    const int soff = s * kSpSlab * (int)ld * 8;
    const bool real = s < nsl;
#pragma unroll
    for (int u = 0; u < kSpPerWave; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(real ? (pk[u] ? rk : rz) : rnone,
                                               (__attribute__((address_space(3))) void*)(buf + loff[u]), 16,
                                               voff[u], soff, 0, 0);
  };
  auto compute = [&](const double* buf) {
    const double* za = buf;
    const double* kb = buf + kSpPart;
#pragma unroll
    for (int k0 = 0; k0 < kSpSlab; k0 += 4) {
      double av[kSlots], bv[kSlots];
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        av[q] = za[(k0 + lk) * kSpCols + 16 * ba[q] + lm];
        bv[q] = kb[(k0 + lk) * kSpCols + 16 * bb[q] + lm];
      }
#pragma unroll
      for (int q = 0; q < kSlots; ++q)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc[q], 0, 0, 0);
    }
  };
  // slab s sits in buffer s % 4; each step waits for its own loads of slab
  // s (two later slabs' loads stay in flight), meets the others at the
  // barrier (after which slab s - 1's buffer is free: every wavefront has
  // consumed it), loads slab s + 3 into that buffer and multiplies slab s
  auto step = [&](int s, double* cur, double* nxt) {
    if (s < nsl) {
      __builtin_amdgcn_s_waitcnt(kWaitVm2Slabs);
      sp_barrier();
      issue(nxt, s + 3);
      compute(cur);
    }
  };
  if (nsl > 0) {
    issue(sp_buf0, 0);
    issue(sp_buf1, 1);
    issue(sp_buf2, 2);
    for (int s0 = 0; s0 < nsl; s0 += 4) {
      step(s0, sp_buf0, sp_buf3);
      step(s0 + 1, sp_buf1, sp_buf0);
      step(s0 + 2, sp_buf2, sp_buf1);
      step(s0 + 3, sp_buf3, sp_buf2);
    }
    // the loads of the slabs past the last one land before the workgroup ends
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
  }
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    if (q < nmine) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = 16 * (bi0 + ba[q]) + lk + 4 * r, gj = 16 * (bj0 + bb[q]) + lm;
        if (gi < d.nu && gj <= gi) d.gpart[((long long)chunk * d.nu + gi) * d.nu + gj] = acc[q][r];
      }
    }
  }
}

template <int kSlots>
__global__ __launch_bounds__(256) void k_stacked_product(DP d, long long per) {
  stacked_product_body<kSlots>((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, d, per);
}



// 1/sqrt(d) for d > 0: the hardware reciprocal square root estimate refined by
// two Newton-Raphson steps r <- r (3 - d r^2) / 2 (quadratic convergence from
// the estimate's accuracy to double precision).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
  double e = fma(-d * r, r, 1.0);
  r = fma(0.5 * r, e, r);
  e = fma(-d * r, r, 1.0);
  return fma(0.5 * r, e, r);
}

// 1/d: the hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r (2 - d r).
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Right-looking blocked Cholesky of the lower triangle of an n x n block held
// in LDS (row-major, leading dimension ld), n a multiple of kPB (callers pad
// with identity rows and columns) and n <= 64 kR, by a workgroup of 64 kWaves
// threads.  Panels of kPB columns: wavefront 0 factorises the panel in
// registers (lane l holds rows jb + l + 64 t; the diagonal row jb + p is in
// lane p).  Inside the panel the elimination runs in the square-root-free
// form A = W D^-1 W^T (column p of W is the updated column p of A, D its
// diagonal): for column p one vector multiply forms every multiplier
// w_qp / d_p in lane q, and readlane broadcasts each to the rows, so the
// chain from one column to the next holds one reciprocal.  The panel's
// columns are then scaled to L = W D^-1/2 together, and its pivots checked
// once.  The inverse of each 16 x 16 diagonal block of L is formed on the way
// and left, transposed, in the block's strict upper triangle (its diagonal is
// 1 / L_aa).  The trailing lower triangle is updated in 16 x 16 tiles on the FP64
// matrix cores (v_mfma_f64_16x16x4f64: A operand lane holds row lane%16,
// k = lane/16; B operand k = lane/16, column lane%16; result register r of a
// lane is row lane/16 + 4 r, column lane%16).
// Returns 0 or the 1-based first column whose pivot is not positive.
constexpr int kPB = 16;

// identity rows n .. np - 1 (columns 0 .. np - 1) below an n x n block in LDS
__device__ __forceinline__ void pad_identity(double* sa, int ld, int n, int np, int t0, int ts) {
  const int cnt = (np - n) * np;
  for (int t = t0; t < cnt; t += ts) {
    const int r = n + t / np, c = t % np;
    sa[r * ld + c] = r == c ? 1.0 : 0.0;
  }
}

template <int kWaves, int kR>
__device__ int chol_blocked_lds(double* sa, int n, int ld, int* sflag) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) *sflag = 0;
  __syncthreads();
  for (int jb = 0; jb < n; jb += kPB) {
    if (wv == 0) {
      double x[kR][kPB];
#pragma unroll
      for (int t = 0; t < kR; ++t) {
        const int r = jb + lane + 64 * t;
#pragma unroll
        for (int p = 0; p < kPB; ++p) x[t][p] = r < n ? sa[r * ld + jb + p] : 0.0;
      }
      double dpiv[kPB];
      // lanes 0..15 also carry row `lane` of the identity through the same
      // column operations, which leaves row r of W_bb^-T D_bb (the inverse
      // of the diagonal block's unit factor, transposed) in lane r
      double y[kPB];
#pragma unroll
      for (int q = 0; q < kPB; ++q) y[q] = q == lane ? 1.0 : 0.0;
      double dv = readlane_d(x[0][0], 0);
#pragma unroll
      for (int p = 0; p < kPB; ++p) {
        dpiv[p] = dv;
        const double m = x[0][p] * rcp_nr(dv);  // lane q: w_qp / d_p
        // the next pivot from lane p + 1's own multiplier: the same operands
        // as its update below, taken first to keep the column chain short
        if (p + 1 < kPB) dv = readlane_d(fma(-x[0][p], m, x[0][p + 1]), p + 1);
#pragma unroll
        for (int q = p + 1; q < kPB; ++q) {
          const double mq = readlane_d(m, q);
#pragma unroll
          for (int t = 0; t < kR; ++t) x[t][q] = fma(-x[t][p], mq, x[t][q]);
          y[q] = fma(-y[p], mq, y[q]);
        }
      }
      int bad = 0;
#pragma unroll
      for (int p = kPB - 1; p >= 0; --p)
        if (!(dpiv[p] > 0.0) || !isfinite(dpiv[p])) bad = jb + p + 1;
      if (bad) {
        if (lane == 0) *sflag = bad;
      } else {
        // L = W D^-1/2 for the whole panel (independent chains); the
        // diagonal block's inverse, (L_bb^-1)[q][r] = y_q(lane r) / sqrt(d_q),
        // goes transposed into the block's strict upper triangle
#pragma unroll
        for (int p = 0; p < kPB; ++p) {
          const double rs = rsqrt_nr(dpiv[p]);
#pragma unroll
          for (int t = 0; t < kR; ++t) {
            const int r = jb + lane + 64 * t;
            if (r < n && jb + p <= r) sa[r * ld + jb + p] = r == jb + p ? dpiv[p] * rs : x[t][p] * rs;
          }
          if (lane < p) sa[(jb + lane) * ld + jb + p] = y[p] * rs;
        }
      }
    }
    __syncthreads();
    if (*sflag) return *sflag;
    const int s0 = jb + kPB, rest = n - s0;
    if (rest <= 0) break;
    const int nt = rest / 16;
    const int lm = lane & 15, lk = lane >> 4;
    int cnt = 0;
    for (int ti = 0; ti < nt; ++ti)
      for (int tl = 0; tl <= ti; ++tl, ++cnt) {
        if (cnt % kWaves != wv) continue;
        const int i0 = s0 + 16 * ti, l0 = s0 + 16 * tl;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < kPB; k0 += 4) {
          const double a = sa[(i0 + lm) * ld + jb + k0 + lk];
          const double b = sa[(l0 + lm) * ld + jb + k0 + lk];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + lk + 4 * r, l = l0 + lm;
          if (l <= i) sa[i * ld + l] -= acc[r];
        }
      }
    __syncthreads();
  }
  return 0;
}

// Factor of an n x n matrix (n <= kSmallN) in one workgroup of 8 wavefronts,
// the matrix padded in LDS to a multiple of 16 with identity rows and its
// lower triangle of 16 x 16 tiles kept there.  Right-looking by 16-column
// panels with look-ahead:
//  - wavefront 0 factorises the panel's diagonal tile in registers
//    (chol_tile16), which also yields the tile's inverse L_kk^-1;
//  - the owner of each block row i below forms L_ik = A_ik L_kk^-T as the
//    product L_kk^-1 A_ik^T on the matrix cores, and after a barrier updates
//    its tiles A_il -= L_ik L_lk^T (l <= i) with the L_ik still in its
//    registers (the accumulator layout of v_mfma_f64_16x16x4f64 is the
//    transpose of its A operand layout, so L_kk^-1 A_ik^T comes out as L_ik
//    in A operand form);
//  - wavefront 0 owns the next block row, so it updates the next diagonal
//    tile first and factorises it while the other wavefronts finish the
//    trailing update: the chain of pivots, the only sequential part, runs
//    behind the matrix-core work.  Two barriers per panel.
// The factorised diagonal tile is staged raw in LDS (rows of W and of
// W^-T D, d_p^-1/2); the block-row owners scale what they read, and the idle
// last wavefront writes the tile's part of A (L and, transposed in its strict
// upper triangle, L_kk^-1) while the others go on.  L_ik goes to A from
// registers as it is formed.  MFMA
// operands: A operand lane holds row lane%16, k = lane/16; B operand k =
// lane/16, column lane%16; result register r row lane/16 + 4 r, column
// lane%16.
constexpr int kCholSmallThreads = 512;
constexpr int kOutWave = kCholSmallThreads / 64 - 1;   // writes the diagonal tiles
// a factorised diagonal tile in LDS: W rows, W^-T D rows (pitch kTileLd),
// d_p^-1/2, d_p; two of them, by panel parity
constexpr int kTileLd = kPB + 1;
constexpr int kRawW = 0, kRawE = kPB * kTileLd, kRawRs = 2 * kPB * kTileLd, kRawD = kRawRs + kPB;
constexpr int kRawSize = kRawD + kPB;

// LDS of k_chol_small: the padded matrix and two staged diagonal tiles
__host__ __device__ inline int chol_small_lds_bytes(int n) {
  const int np = (n + kPB - 1) / kPB * kPB;
  return 8 * (np * (np + 1) + 2 * kRawSize);
}

// LDL^T of one 16 x 16 symmetric tile by lanes 0..15 of one wavefront, in the
// square-root-free column form A = W D^-1 W^T: lane r holds row r of the tile
// (x[q] = A[r][q]) and row r of the identity (y), and each column p is
// eliminated from the later ones, x[q] -= x[p] w_qp / d_p (y alike), the
// multiplier w_qp / d_p formed in lane q and broadcast along the row of lanes.
// At the end lane r holds row r of W in x and row r of W^-T D in y.  The
// pivot chain holds only what the next pivot needs: d_p+1 = a_p+1,p+1 -
// w_p+1,p^2 / d_p from the reciprocal estimate r0 of d_p and its error
// e = 1 - d_p r0, 1/d_p = r0 (1 + e + e^2 + e^3 + ...) (the estimate is good
// to about 2^-24, so three terms leave less than 2^-90).  Lane p of dpv
// receives d_p.
// updates x[q], y[q] for kLo <= q < kHi by column P with multipliers m
template <int P, int kLo, int kHi, int... Q>
__device__ __forceinline__ void tile_eliminate(double (&x)[kPB], double (&y)[kPB], double m,
                                               std::integer_sequence<int, Q...>) {
  const double nx = -x[P], ny = -y[P];
  auto one = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    if constexpr (q > P && q >= kLo && q < kHi) {
      const double mq = row_bcast<q>(m);
      x[q] = fma(mq, nx, x[q]);
      y[q] = fma(mq, ny, y[q]);
      // y is read only at the end: pin its update here so that it is not
      // sunk there, which would keep every broadcast multiplier alive
      asm volatile("" : "+v"(y[q]));
    }
  };
  (one(std::integral_constant<int, Q>{}), ...);
}

// Step P in one scheduling region with the rest of step P - 1: its pivot
// chain first, then the rest (the tail) of step P - 1, then its own first two
// columns (the head, all the next step's chain needs); no instruction moves
// across regions, which keeps the broadcasts from being hoisted into a
// register pile-up.
template <int P>
__device__ __forceinline__ void tile_chain(double (&x)[kPB], double (&y)[kPB], double d, double mprev,
                                           double& dpv, int lane) {
  constexpr auto all = std::make_integer_sequence<int, kPB>{};
  dpv = lane == P ? d : dpv;
  const double r0 = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, r0, 1.0);
  const double t = fma(e, fma(e, e, e), e);
  const double m = x[P] * fma(r0, t, r0);
  double dn = 0.0;
  if constexpr (P + 1 < kPB) {
    const double a = x[P] * x[P] * r0;
    dn = row_bcast<P + 1>(fma(-a, t, x[P + 1] - a));
  }
  if constexpr (P > 0) tile_eliminate<P - 1, P + 2, kPB>(x, y, mprev, all);
  tile_eliminate<P, P + 1, P + 3>(x, y, m, all);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (P + 1 < kPB) tile_chain<P + 1>(x, y, dn, m, dpv, lane);
}

// Pivot test of a factorised diagonal tile at jb, then lane r < 16 stages row
// r of W and of W^-T D, d_r^-1/2 and d_r in raw.  Returns the 1-based first
// column whose pivot is not positive (then nothing is staged), else 0.
__device__ __forceinline__ int chol_tile16_stage(const double (&x)[kPB], const double (&y)[kPB], double dpv,
                                                 int jb, double* raw, int lane) {
  const unsigned long long badl = __ballot(lane < kPB && !(dpv > 0.0 && isfinite(dpv)));
  if (badl) return jb + __ffsll((long long)badl);
  if (lane < kPB) {
#pragma unroll
    for (int q = 0; q < kPB; ++q) {
      raw[kRawW + lane * kTileLd + q] = x[q];
      raw[kRawE + lane * kTileLd + q] = y[q];
    }
    raw[kRawRs + lane] = rsqrt_nr(dpv);
    raw[kRawD + lane] = dpv;
  }
  return 0;
}

// A's part of the staged diagonal tile at jb, by one wavefront: row jb + r,
// L[jb + r][jb + p] = W[r][p] d_p^-1/2 (p <= r) and, in the strict upper
// part, the inverse's transpose (L^-1)[p][r] = d_p^-1/2 (W^-T D)[r][p].
__device__ __forceinline__ void chol_tile16_write(const double* raw, double* A, int n, int jb, int lane) {
#pragma unroll
  for (int u = 0; u < kPB * kPB / 64; ++u) {
    const int t = lane + 64 * u, r = t / kPB, p = t % kPB;
    if (jb + r < n && jb + p < n) {
      const double rs = raw[kRawRs + p];
      const double v = p < r ? raw[kRawW + r * kTileLd + p] * rs
                             : (p == r ? raw[kRawD + p] * rs : raw[kRawE + r * kTileLd + p] * rs);
      A[(long long)(jb + r) * n + jb + p] = v;
    }
  }
}

__device__ __forceinline__ void chol_small_body(int bx_, int by_, int gx_, const double* src, double* A, int n,
                                                                   int* info) {
  extern __shared__ double sa[];
  __shared__ int sflag;
  const int np = (n + kPB - 1) / kPB * kPB, nb = np / kPB;
  const int ld = np + 1, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  double* raw = sa + np * ld;   // two staged diagonal tiles, by panel parity
  double x[kPB], y[kPB], dpv = 0.0;
  if (tid == 0) sflag = 0;
  if (wv == 0) {
    // panel 0's diagonal tile straight from global memory
#pragma unroll
    for (int q = 0; q < kPB; ++q) {
      x[q] = lane < n && q < n ? src[(long long)lane * n + q] : (lane == q ? 1.0 : 0.0);
      y[q] = lane == q ? 1.0 : 0.0;
    }
  } else {
    // the other wavefronts stage the lower block triangle below tile row 0:
    // tile tau of block row bi >= 1, block column bl <= bi, in row-major order
    const int ntile = (nb - 1) * (nb + 2) / 2, total = ntile * kPB * kPB;
    const int start = tid - 64, stride = kCholSmallThreads - 64;
    for (int t0 = start; t0 < total; t0 += kStageBatch * stride) {
      double v[kStageBatch];
      int o[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int t = t0 + u * stride;
        o[u] = -1;
        if (t < total) {
          int tau = t / (kPB * kPB), bi = 1;
          while (tau >= bi + 1) tau -= ++bi;
          const int e = t % (kPB * kPB);
          const int i = kPB * bi + e / kPB, c = kPB * tau + e % kPB;
          v[u] = i < n && c < n ? src[(long long)i * n + c] : (i == c ? 1.0 : 0.0);
          o[u] = i * ld + c;
        }
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u)
        if (o[u] >= 0) sa[o[u]] = v[u];
    }
  }
  if (wv == 0) {
    tile_chain<0>(x, y, row_bcast<0>(x[0]), 0.0, dpv, lane);
    const int bad = chol_tile16_stage(x, y, dpv, 0, raw, lane);
    if (bad && lane == 0) sflag = bad;
  }
  __syncthreads();
  for (int k = 0; k + 1 < nb && sflag == 0; ++k) {
    const int jb = kPB * k;
    const double* rk = raw + (k & 1) * kRawSize;
    if (wv == kOutWave) chol_tile16_write(rk, A, n, jb, lane);
    // block row owned by this wavefront: k + 1 for wavefront 0, k + 1 + wv
    // for the others (nb <= 8 leaves the last wavefront idle)
    const int i = k + 1 + wv;
    const bool own = i < nb;
    v4d li = {0.0, 0.0, 0.0, 0.0};
    if (own) {
      const int i0 = kPB * i;
      // (L_kk^-1)[lm][c] = d_lm^-1/2 (W^-T D)[c][lm]
      const double rsl = rk[kRawRs + lm];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double m1 = rsl * rk[kRawE + (4 * j + lk) * kTileLd + lm];
        const double b = sa[(i0 + lm) * ld + jb + 4 * j + lk];
        li = __builtin_amdgcn_mfma_f64_16x16x4f64(m1, b, li, 0, 0, 0);
      }
      // register r: L[i0 + lm][jb + lk + 4 r]
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sa[(i0 + lm) * ld + jb + lk + 4 * r] = li[r];
        if (i0 + lm < n && jb + lk + 4 * r < n) A[(long long)(i0 + lm) * n + jb + lk + 4 * r] = li[r];
      }
    }
    __syncthreads();
    if (own) {
      const int i0 = kPB * i;
      // wavefront 0 has only the diagonal tile (k+1, k+1); the others go
      // from their diagonal tile leftwards
      for (int l = i; l > k; --l) {
        const int l0 = kPB * l;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double b = sa[(l0 + lm) * ld + jb + 4 * j + lk];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(li[j], b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sa[(i0 + lk + 4 * r) * ld + l0 + lm] -= acc[r];
      }
    }
    if (wv == 0) {
      wave_sync();
      const int j1 = jb + kPB;
#pragma unroll
      for (int q = 0; q < kPB; ++q) {
        x[q] = lane < kPB ? sa[(j1 + lane) * ld + j1 + q] : 0.0;
        y[q] = lane == q ? 1.0 : 0.0;
      }
      tile_chain<0>(x, y, row_bcast<0>(x[0]), 0.0, dpv, lane);
      const int bad = chol_tile16_stage(x, y, dpv, j1, raw + ((k + 1) & 1) * kRawSize, lane);
      if (bad && lane == 0) sflag = bad;
    }
    __syncthreads();
  }
  if (sflag == 0 && wv == kOutWave) chol_tile16_write(raw + ((nb - 1) & 1) * kRawSize, A, n, kPB * (nb - 1), lane);
  if (tid == 0) *info = sflag;
}

__global__ __launch_bounds__(kCholSmallThreads) void k_chol_small(const double* src, double* A, int n,
                                                                   int* info) {
  chol_small_body((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, src, A, n, info);
}

// blocked: factor the 64 x 64 diagonal block at jb
__device__ __forceinline__ void chol_diag_body(int bx_, int by_, int gx_, double* A, int n, int jb, int* info) {
  if (*info != 0) return;
  __shared__ double sa[kNB * (kNB + 1)];
  __shared__ int sflag;
  const int nb = min(kNB, n - jb), ld = kNB + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nbp = (nb + kPB - 1) / kPB * kPB;
  copy2d_overlapped(sa, ld, A + (long long)jb * n + jb, n, nb, nb, threadIdx.x, kThreads);
  pad_identity(sa, ld, nb, nbp, threadIdx.x, kThreads);
  __syncthreads();
  const int r = chol_blocked_lds<kWavesD, 1>(sa, nbp, ld, &sflag);
  for (int i = wv; i < nb; i += kWavesD)
    for (int l = lane; l <= i; l += 64) A[(long long)(jb + i) * n + jb + l] = sa[i * ld + l];
  if (threadIdx.x == 0 && r) *info = jb + r;
}

__global__ __launch_bounds__(kThreads) void k_chol_diag(double* A, int n, int jb, int* info) {
  chol_diag_body((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, A, n, jb, info);
}

// blocked: A[i, jb:jb+nb] <- A[i, jb:jb+nb] L_jj^-T for rows below the block.
// A wavefront takes one row at a time with lane q holding column q; lane q
// keeps row q of L_jj in registers, so the forward substitution is 64
// readlane broadcasts and fused multiply-adds with no memory traffic.
constexpr int kTrsmRowsPerWave = 4;

__device__ __forceinline__ void chol_trsm_body(int bx_, int by_, int gx_, double* A, int n, int jb, const int* info) {
  if (*info != 0) return;
  __shared__ double sinv[kNB];
  const int nb = min(kNB, n - jb);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double lrow[kNB];
#pragma unroll
  for (int p = 0; p < kNB; ++p)
    lrow[p] = (lane < nb && p <= lane) ? A[(long long)(jb + lane) * n + jb + p] : 0.0;
  if (threadIdx.x < kNB)
    sinv[threadIdx.x] = threadIdx.x < nb ? 1.0 / A[(long long)(jb + threadIdx.x) * n + jb + threadIdx.x] : 0.0;
  __syncthreads();
  const int rows = n - jb - nb;
  for (int r = bx_ * kWavesD + wv; r < rows; r += gx_ * kWavesD) {
    double* row = A + (long long)(jb + nb + r) * n + jb;
    double v = lane < nb ? row[lane] : 0.0;
#pragma unroll
    for (int p = 0; p < kNB; ++p) {
      if (p < nb) {
        const double xp = readlane_d(v, p) * sinv[p];
        if (lane == p) v = xp;
        else if (lane > p) v = fma(-xp, lrow[p], v);
      }
    }
    if (lane < nb) row[lane] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_chol_trsm(double* A, int n, int jb, const int* info) {
  chol_trsm_body((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, A, n, jb, info);
}

// blocked: trailing update A[i, l] -= sum_p A[i, p] A[l, p] over the lower
// 64 x 64 tiles, on the FP64 matrix cores.  Each of the 4 waves owns a 32 x 32
// quarter as 2 x 2 blocks of v_mfma_f64_16x16x4f64 (A operand: lane holds
// row lane%16, k = lane/16; B operand: k = lane/16, column lane%16; result
// register r of a lane: row lane/16 + 4 r, column lane%16).

__device__ __forceinline__ void chol_update_body(int bx_, int by_, int gx_, double* A, int n, int jb, const int* info) {
  if (*info != 0) return;
  const int nb = min(kNB, n - jb);
  const int s0 = jb + nb;
  const int ti = by_, tl = bx_;
  if (tl > ti) return;
  const int i0 = s0 + ti * 64, l0 = s0 + tl * 64;
  __shared__ double sa[64][kNB + 1];
  __shared__ double sb[64][kNB + 1];
  for (int t = threadIdx.x; t < 64 * kNB; t += blockDim.x) {
    const int r = t / kNB, p = t % kNB;
    const bool kin = p < nb;
    sa[r][p] = (kin && i0 + r < n) ? A[(long long)(i0 + r) * n + jb + p] : 0.0;
    sb[r][p] = (kin && l0 + r < n) ? A[(long long)(l0 + r) * n + jb + p] : 0.0;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb = (wv >> 1) * 32, cb = (wv & 1) * 32;   // wave's quarter
  const int lm = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kNB; k0 += 4) {
    const double a0 = sa[rb + lm][k0 + lk], a1 = sa[rb + 16 + lm][k0 + lk];
    const double b0 = sb[cb + lm][k0 + lk], b1 = sb[cb + 16 + lm][k0 + lk];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + rb + 16 * a + lk + 4 * r, l = l0 + cb + 16 * b + lm;
        if (i < n && l <= i) A[(long long)i * n + l] -= acc[a][b][r];
      }
}

__global__ __launch_bounds__(kThreads) void k_chol_update(double* A, int n, int jb, const int* info) {
  chol_update_body((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, A, n, jb, info);
}

// p_u = K_hat^-1 rhs with rhs = -r1u + sum_i rpart_i, from the Cholesky
// factor L (lower triangle of `L`, row-major).  One workgroup of kRThreads
// (16 wavefronts).  The right-hand side is summed over scenarios in a fixed
// order (wavefront w takes a contiguous 1/16 of the scenarios, partial sums
// added in wavefront order).  Both triangular solves go by blocks of 16 rows:
// the off-diagonal part is a matrix-vector product (one wavefront per row of
// the block for L, per column for L^T, lanes over the long dimension, then a
// shuffle reduction), and the 16 x 16 diagonal triangle is solved by one
// wavefront in registers (lane r holds unknown r; readlane broadcasts).
// kLDS: L staged in LDS (leading dimension n + 1); else read from global.
constexpr int kRB = 16, kRThreads = 1024, kRWaves = kRThreads / 64;

// the reduced solve stages L in LDS when it fits next to its reduction buffer
__host__ __device__ inline bool rsolve_lds(int n) {
  return 8LL * ((long long)n * (n + 1) + n) + 8LL * kRWaves * 64 <= 160 * 1024;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <bool kLDS>
__device__ __forceinline__ void reduced_solve_body(int bx_, int by_, int gx_, const DP& d, const double* r1u, const double* Lg,
                                                             double* pu) {
  extern __shared__ double sm[];
  __shared__ double red[kRWaves][64];
  const int n = d.nu, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ld = kLDS ? n + 1 : n;
  double* y = sm;
  const double* L = Lg;
  if (kLDS) {
    double* sl = sm + n;
    copy2d_overlapped(sl, ld, Lg, n, n, n, tid, kRThreads);
    L = sl;
  }
  // right-hand side
  const int per = (d.N + kRWaves - 1) / kRWaves;
  const int k0 = wv * per, k1 = min(d.N, k0 + per);
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int c = c0 + lane;
    double acc = 0.0;
    if (c < n) {
      // loads in batches of 8 so that they are in flight together
      int k = k0;
      for (; k + 8 <= k1; k += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = d.rpart[(long long)(k + u) * n + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
      }
      for (; k < k1; ++k) acc += d.rpart[(long long)k * n + c];
    }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && c < n) {
      double sum = -r1u[c];
      for (int q = 0; q < kRWaves; ++q) sum += red[q][lane];
      y[c] = sum;
    }
    __syncthreads();
  }
  // forward: L y = b
  for (int jb = 0; jb < n; jb += kRB) {
    const int nb = min(kRB, n - jb);
    if (wv < nb) {
      const double* row = L + (long long)(jb + wv) * ld;
      double acc = 0.0;
      for (int q = lane; q < jb; q += 64) acc = fma(row[q], y[q], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[jb + wv] -= acc;
    }
    __syncthreads();
    if (wv == 0) {
      const int r = lane;
      double lrow[kRB];
#pragma unroll
      for (int p = 0; p < kRB; ++p) lrow[p] = (r < nb && p <= r) ? L[(long long)(jb + r) * ld + jb + p] : 0.0;
      const double myinv = r < nb ? rcp_nr(L[(long long)(jb + r) * ld + jb + r]) : 0.0;  // 1/L_rr
      double v = r < nb ? y[jb + r] : 0.0;
#pragma unroll
      for (int p = 0; p < kRB; ++p) {
        if (p < nb) {
          const double vp = readlane_d(v, p) * readlane_d(myinv, p);
          if (r == p) v = vp;
          else if (r > p) v = fma(-lrow[p], vp, v);
        }
      }
      if (r < nb) y[jb + r] = v;
    }
    __syncthreads();
  }
  // backward: L^T x = y
  for (int jb = ((n - 1) / kRB) * kRB; jb >= 0; jb -= kRB) {
    const int nb = min(kRB, n - jb);
    if (wv < nb) {
      double acc = 0.0;
      for (int i = jb + nb + lane; i < n; i += 64) acc = fma(L[(long long)i * ld + jb + wv], y[i], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[jb + wv] -= acc;
    }
    __syncthreads();
    if (wv == 0) {
      const int r = lane;
      // lane r holds column r of the diagonal block: L[jb + p][jb + r], p >= r
      double lcol[kRB];
#pragma unroll
      for (int p = 0; p < kRB; ++p) lcol[p] = (r < nb && p < nb && p >= r) ? L[(long long)(jb + p) * ld + jb + r] : 0.0;
      const double myinv = r < nb ? rcp_nr(L[(long long)(jb + r) * ld + jb + r]) : 0.0;
      double v = r < nb ? y[jb + r] : 0.0;
#pragma unroll
      for (int p = kRB - 1; p >= 0; --p) {
        if (p < nb) {
          const double vp = readlane_d(v, p) * readlane_d(myinv, p);
          if (r == p) v = vp;
          else if (r < p) v = fma(-lcol[p], vp, v);
        }
      }
      if (r < nb) y[jb + r] = v;
    }
    __syncthreads();
  }
  for (int c = tid; c < n; c += kRThreads) pu[c] = y[c];
}

template <bool kLDS>
__global__ __launch_bounds__(kRThreads) void k_reduced_solve(DP d, const double* r1u, const double* Lg,
                                                             double* pu) {
  reduced_solve_body<kLDS>((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, d, r1u, Lg, pu);
}

// Reduced solve with the factor stored by k_chol_small.  Every wavefront
// stages the lower block triangle of the factor (16 x 16 tiles, zeros past
// n) into LDS while summing the scenario parts of the right-hand side.  Then
// block substitution, right-looking with look-ahead, one barrier per block:
// after block j is solved, the owner of each later block i subtracts
// L_ij y_j (lane = row, four column quarters combined by two shuffles);
// wavefront 0 owns block j + 1, so it updates it first and solves it at once
// with the block's stored inverse (y_r = t_r / L_rr + sum_{p<r}
// (L^-1)[r][p] t_p, t broadcast along the row of 16 lanes with DPP).  The
// backward pass runs the same way on the transposed tiles.
constexpr int kIThreads = 512, kIWaves = kIThreads / 64;
constexpr int kRhsPre = 16;   // scenarios per wavefront whose parts are loaded ahead

__host__ __device__ inline long long rsolve_blk_lds_bytes(int n) {
  const long long np = (n + 15) / 16 * 16;
  return 8LL * (np * (np + 1) + 2 * np);
}

// y[b0 + r] <- the block's inverse (kFwd: L_bb^-1, else L_bb^-T) applied to
// y[b0 .. b0 + 15], by one wavefront (lanes 0..15 write)
template <bool kFwd, int... P>
__device__ __forceinline__ void rsolve_diag(const double* sa, int ld, const double* rd, double* y, int b0,
                                            int lane, std::integer_sequence<int, P...>) {
  const int r = lane & 15;
  double c[kPB];
  // (L^-1)[r][p] (p < r) is stored at [b0 + p][b0 + r], (L^-1)[p][r] (p > r)
  // at [b0 + r][b0 + p]
  ((c[P] = kFwd ? (P < r ? sa[(b0 + P) * ld + b0 + r] : 0.0) : (P > r ? sa[(b0 + r) * ld + b0 + P] : 0.0)), ...);
  const double t = y[b0 + r];
  double a0 = rd[b0 + r] * t, a1 = 0.0;
  ((P % 2 == 0 ? (a0 = fma(c[P], row_bcast<P>(t), a0)) : (a1 = fma(c[P], row_bcast<P>(t), a1))), ...);
  wave_sync();
  if (lane < kPB) y[b0 + r] = a0 + a1;
}

// y_i -= L_ij y_j (kFwd) or L_ji^T y_j, 16 x 16, by one wavefront
template <bool kFwd>
__device__ __forceinline__ void rsolve_update(const double* sa, int ld, double* y, int i0, int j0, int lane) {
  const int r = lane & 15, g = lane >> 4;
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = g + 4 * u;
    const double l = kFwd ? sa[(i0 + r) * ld + j0 + c] : sa[(j0 + c) * ld + i0 + r];
    acc = fma(l, y[j0 + c], acc);
  }
  acc += __shfl_xor(acc, 16);
  acc += __shfl_xor(acc, 32);
  if (g == 0) y[i0 + r] -= acc;
}

__device__ __forceinline__ void reduced_solve_blk_body(int bx_, int by_, int gx_, const DP& d, const double* r1u,
                                                                 const double* A, double* pu) {
  extern __shared__ double sm[];
  __shared__ double red[kIThreads];
  const int n = d.nu, np = (n + kPB - 1) / kPB * kPB, nb = np / kPB, ld = np + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* sa = sm;
  double* y = sa + (long long)np * ld;
  double* rd = y + np;
  // the right-hand side's loads first (up to kRhsPre scenarios of each of
  // the two column chunks per lane), in flight during the staging
  const int per = (d.N + kIWaves - 1) / kIWaves;
  const int k0 = wv * per, k1 = min(d.N, k0 + per);
  double pre[2][kRhsPre];
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const int c = 64 * ch + lane;
#pragma unroll
    for (int u = 0; u < kRhsPre; ++u)
      pre[ch][u] = c < n && k0 + u < k1 ? d.rpart[(long long)(k0 + u) * n + c] : 0.0;
  }
  {
    // lower block triangle: tile tau of block row bi, block column bl <= bi,
    // in row-major order
    const int total = nb * (nb + 1) / 2 * kPB * kPB;
    for (int t0 = tid; t0 < total; t0 += kStageBatch * kIThreads) {
      double v[kStageBatch];
      int o[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int t = t0 + u * kIThreads;
        o[u] = -1;
        if (t < total) {
          int tau = t / (kPB * kPB), bi = 0;
          while (tau >= bi + 1) tau -= ++bi;
          const int e = t % (kPB * kPB);
          const int i = kPB * bi + e / kPB, c = kPB * tau + e % kPB;
          v[u] = i < n && c < n ? A[(long long)i * n + c] : 0.0;
          o[u] = i * ld + c;
        }
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u)
        if (o[u] >= 0) sa[o[u]] = v[u];
    }
  }
  // right-hand side: sum of the scenario parts, scenario slices per
  // wavefront, each slice in scenario order
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const int c0 = 64 * ch, c = c0 + lane;
    if (c0 >= np) break;
    double acc = 0.0;
    if (c < n) {
#pragma unroll
      for (int u = 0; u < kRhsPre; ++u)
        if (k0 + u < k1) acc += pre[ch][u];
      for (int k = k0 + kRhsPre; k < k1; ++k) acc += d.rpart[(long long)k * n + c];
    }
    red[wv * 64 + lane] = acc;
    __syncthreads();
    if (wv == 0 && c < np) {
      double sum = c < n ? -r1u[c] : 0.0;
      for (int q = 0; q < kIWaves; ++q) sum += red[q * 64 + lane];
      y[c] = sum;
    }
    __syncthreads();
  }
  for (int c = tid; c < np; c += kIThreads) rd[c] = c < n ? rcp_nr(sa[c * ld + c]) : 0.0;
  __syncthreads();
  constexpr auto all = std::make_integer_sequence<int, kPB>{};
  // forward: L y = b
  if (wv == 0) rsolve_diag<true>(sa, ld, rd, y, 0, lane, all);
  __syncthreads();
  for (int j = 0; j + 1 < nb; ++j) {
    const int i = j + 1 + wv;
    if (i < nb) rsolve_update<true>(sa, ld, y, kPB * i, kPB * j, lane);
    if (wv == 0) {
      wave_sync();
      rsolve_diag<true>(sa, ld, rd, y, kPB * (j + 1), lane, all);
    }
    __syncthreads();
  }
  // backward: L^T x = y, x overwriting y
  if (wv == 0) rsolve_diag<false>(sa, ld, rd, y, kPB * (nb - 1), lane, all);
  __syncthreads();
  for (int j = nb - 1; j > 0; --j) {
    const int i = j - 1 - wv;
    if (i >= 0) rsolve_update<false>(sa, ld, y, kPB * i, kPB * j, lane);
    if (wv == 0) {
      wave_sync();
      rsolve_diag<false>(sa, ld, rd, y, kPB * (j - 1), lane, all);
    }
    __syncthreads();
  }
  for (int c = tid; c < n; c += kIThreads) pu[c] = y[c];
}

__global__ __launch_bounds__(kIThreads) void k_reduced_solve_blk(DP d, const double* r1u,
                                                                 const double* A, double* pu) {
  reduced_solve_blk_body((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, d, r1u, A, pu);
}

}  // namespace

// raise the dynamic LDS limit of a kernel to what this problem needs (never lowered)
static hipError_t allow_lds(const void* fn, int* cur, int need) {
  if (need <= *cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, need);
  if (e == hipSuccess) *cur = need;
  return e;
}

hipError_t configure_dense_kernels(const DP& d) {
  static int c1 = 0, c2 = 0, c3 = 0, c5 = 0;
  hipError_t e = hipSuccess;
  if (d.nu <= kSmallN) e = allow_lds((const void*)k_chol_small, &c1, chol_small_lds_bytes(d.nu));
  if (e == hipSuccess && d.nu <= kSmallN)
    e = allow_lds((const void*)k_reduced_solve_blk, &c5, (int)rsolve_blk_lds_bytes(d.nu));
  if (e == hipSuccess && d.nu > kSmallN) {
    if (rsolve_lds(d.nu))
      e = allow_lds((const void*)k_reduced_solve<true>, &c2, 8 * (d.nu * (d.nu + 1) + d.nu));
    else
      e = allow_lds((const void*)k_reduced_solve<false>, &c3, 8 * d.nu);
  }
  return e;
}

__device__ __forceinline__ void copy_body(int bx_, int by_, int gx_, const double* a, double* b, long long n) {
  long long t = (long long)bx_ * blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

__global__ void k_copy(const double* a, double* b, long long n) {
  copy_body((int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, a, b, n);
}

void launch_copy(const double* a, double* b, long long n, hipStream_t s) {
  k_copy<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(a, b, n);
}

void launch_scenario_sum(const DP& d, const double* su, double dw, double* khat, hipStream_t s) {
  const long long ntri = (long long)d.nu * (d.nu + 1) / 2;
  const double* src = d.variant == 2 ? d.gpart : d.part;
  const int cnt = d.variant == 2 ? d.nchunk : d.N;
  if (cnt >= kSumManyFrom) {
    const unsigned grid = (unsigned)((ntri + kSumEntriesMany - 1) / kSumEntriesMany);
    k_sym_sum<kSumEntriesMany, kSumWavesMany><<<grid, kSumEntriesMany * kSumWavesMany, 0, s>>>(d, src, cnt, su, dw,
                                                                                                khat);
  } else {
    const unsigned grid = (unsigned)((ntri + kSumEntries - 1) / kSumEntries);
    k_sym_sum<kSumEntries, kSumWaves><<<grid, kSumEntries * kSumWaves, 0, s>>>(d, src, cnt, su, dw, khat);
  }
}

void launch_stacked_product(const DP& d, hipStream_t s) {
  const int T = sp_nsuper(d.nu), nblk = sp_nblk(d.nu);
  const long long per = sp_rows_per_chunk((long long)d.N * d.nz, d.nchunk);
  // blocks per wavefront: the largest super-tile's count over 4 wavefronts
  const int most = nblk > kSB ? kSB * kSB : nblk * (nblk + 1) / 2;
  const int slots = (most + 3) / 4;
  const dim3 grid(T * (T + 1) / 2, d.nchunk);
  if (slots <= 1) k_stacked_product<1><<<grid, 256, 0, s>>>(d, per);
  else if (slots <= 2) k_stacked_product<2><<<grid, 256, 0, s>>>(d, per);
  else if (slots <= 4) k_stacked_product<4><<<grid, 256, 0, s>>>(d, per);
  else if (slots <= 7) k_stacked_product<7><<<grid, 256, 0, s>>>(d, per);
  else k_stacked_product<kSBMax><<<grid, 256, 0, s>>>(d, per);
}

void launch_cholesky_from(const DP& d, const double* src, double* a, int* info, hipStream_t s) {
  const int n = d.nu;
  if (n <= kSmallN) {
    k_chol_small<<<1, kCholSmallThreads, (size_t)chol_small_lds_bytes(n), s>>>(src, a, n, info);
    return;
  }
  if (src != a) launch_copy(src, a, (long long)n * n, s);
  k_set_int<<<1, 1, 0, s>>>(info, 0);
  for (int jb = 0; jb < n; jb += kNB) {
    k_chol_diag<<<1, kThreads, 0, s>>>(a, n, jb, info);
    const int nb = n - jb < kNB ? n - jb : kNB;
    const int rest = n - jb - nb;
    if (rest <= 0) break;
    k_chol_trsm<<<(rest + kWavesD * kTrsmRowsPerWave - 1) / (kWavesD * kTrsmRowsPerWave), kThreads, 0, s>>>(
        a, n, jb, info);
    const int nt = (rest + 63) / 64;
    k_chol_update<<<dim3(nt, nt), kThreads, 0, s>>>(a, n, jb, info);
  }
}

void launch_cholesky(const DP& d, double* a, int* info, hipStream_t s) {
  launch_cholesky_from(d, a, a, info, s);
}

void launch_reduced_solve(const DP& d, const double* r1u, const double* chol, double* pu,
                          hipStream_t s) {
  if (d.nu <= kSmallN)
    k_reduced_solve_blk<<<1, kIThreads, (size_t)rsolve_blk_lds_bytes(d.nu), s>>>(d, r1u, chol, pu);
  else if (rsolve_lds(d.nu))
    k_reduced_solve<true><<<1, kRThreads, 8 * ((size_t)d.nu * (d.nu + 1) + d.nu), s>>>(d, r1u, chol, pu);
  else
    k_reduced_solve<false><<<1, kRThreads, 8 * (size_t)d.nu, s>>>(d, r1u, chol, pu);
}

// ---- several instances in one launch (block b is block (blk[b].bx, blk[b].by)
// of instance blk[b].inst's own grid, blk[b].gx wide)
#define RKKT_MULTI_ARGS \
  const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its, const MultiBlk* __restrict__ blk
#define RKKT_MULTI_PROLOGUE                          \
  const MultiBlk mb = blk[blockIdx.x];               \
  const DP& d = dps[mb.inst];                        \
  const rkkt_iteration& it = its[mb.inst];     \
  (void)it;

__global__ __launch_bounds__(kSumEntries * kSumWaves) void k_sym_sum_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  sym_sum_body<kSumEntries, kSumWaves>(mb.bx, d, d.variant == 2 ? d.gpart : d.part,
                                       d.variant == 2 ? d.nchunk : d.N, it.sigma_u, it.delta_w, it.khat);
}
template <int kSlots>
__global__ __launch_bounds__(256) void k_stacked_product_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  stacked_product_body<kSlots>(mb.bx, mb.by, mb.gx, d, sp_rows_per_chunk((long long)d.N * d.nz, d.nchunk));
}
__global__ __launch_bounds__(kCholSmallThreads) void k_chol_small_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  chol_small_body(mb.bx, mb.by, mb.gx, it.khat, it.chol, d.nu, it.info);
}
__global__ void k_copy_chol_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  copy_body(mb.bx, mb.by, mb.gx, it.khat, it.chol, (long long)d.nu * d.nu);
}
__global__ void k_set_info_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  (void)d;
  if (threadIdx.x == 0) *it.info = 0;
}
__global__ __launch_bounds__(kThreads) void k_chol_diag_m(RKKT_MULTI_ARGS, int jb) {
  RKKT_MULTI_PROLOGUE
  chol_diag_body(mb.bx, mb.by, mb.gx, it.chol, d.nu, jb, it.info);
}
__global__ __launch_bounds__(kThreads) void k_chol_trsm_m(RKKT_MULTI_ARGS, int jb) {
  RKKT_MULTI_PROLOGUE
  chol_trsm_body(mb.bx, mb.by, mb.gx, it.chol, d.nu, jb, it.info);
}
__global__ __launch_bounds__(kThreads) void k_chol_update_m(RKKT_MULTI_ARGS, int jb) {
  RKKT_MULTI_PROLOGUE
  chol_update_body(mb.bx, mb.by, mb.gx, it.chol, d.nu, jb, it.info);
}
template <bool kLDS>
__global__ __launch_bounds__(kRThreads) void k_reduced_solve_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  reduced_solve_body<kLDS>(mb.bx, mb.by, mb.gx, d, it.r1u, it.chol, it.pu);
}
__global__ __launch_bounds__(kIThreads) void k_reduced_solve_blk_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  reduced_solve_blk_body(mb.bx, mb.by, mb.gx, d, it.r1u, it.chol, it.pu);
}

static int stacked_slots_variant(const DP& d) {
  const int nblk = sp_nblk(d.nu);
  const int most = nblk > kSB ? kSB * kSB : nblk * (nblk + 1) / 2;
  const int slots = (most + 3) / 4;
  return slots <= 1 ? 0 : slots <= 2 ? 1 : slots <= 4 ? 2 : slots <= 7 ? 3 : 4;
}

// the launches of launch_stacked_product (stacked variant), launch_scenario_sum,
// launch_cholesky_from (K_hat into the factor) and launch_reduced_solve
void launches_dense(const DP& d, std::vector<Launch>& out) {
  const int n = d.nu;
  if (d.variant == 2) {
    const int T = sp_nsuper(n);
    out.push_back(Launch{kStStacked * 4096, kKStacked, stacked_slots_variant(d), T * (T + 1) / 2, d.nchunk, 256,
                         0, 0});
  }
  const long long ntri = (long long)n * (n + 1) / 2;
  out.push_back(Launch{kStSum * 4096, kKSymSum, 0, (int)((ntri + kSumEntries - 1) / kSumEntries), 1,
                       kSumEntries * kSumWaves, 0, 0});
  const int F = kStFactor * 4096;
  if (n <= kSmallN) {
    out.push_back(Launch{F, kKCholSmall, 0, 1, 1, kCholSmallThreads, 0, chol_small_lds_bytes(n)});
  } else {
    out.push_back(Launch{F, kKCopyChol, 0, (int)(((long long)n * n + kThreads - 1) / kThreads), 1, kThreads, 0, 0});
    out.push_back(Launch{F + 1, kKSetInfo, 0, 1, 1, 1, 0, 0});
    for (int jb = 0, q = 0; jb < n; jb += kNB, ++q) {
      out.push_back(Launch{F + 2 + 3 * q, kKCholDiag, 0, 1, 1, kThreads, jb, 0});
      const int nb = n - jb < kNB ? n - jb : kNB;
      const int rest = n - jb - nb;
      if (rest <= 0) break;
      out.push_back(Launch{F + 3 + 3 * q, kKCholTrsm, 0,
                           (rest + kWavesD * kTrsmRowsPerWave - 1) / (kWavesD * kTrsmRowsPerWave), 1, kThreads, jb,
                           0});
      const int nt = (rest + 63) / 64;
      out.push_back(Launch{F + 4 + 3 * q, kKCholUpdate, 0, nt, nt, kThreads, jb, 0});
    }
  }
  if (n <= kSmallN)
    out.push_back(Launch{kStRSolve * 4096, kKRSolveBlk, 0, 1, 1, kIThreads, 0, rsolve_blk_lds_bytes(n)});
  else if (rsolve_lds(n))
    out.push_back(Launch{kStRSolve * 4096, kKRSolve, 1, 1, 1, kRThreads, 0, 8LL * ((long long)n * (n + 1) + n)});
  else
    out.push_back(Launch{kStRSolve * 4096, kKRSolve, 0, 1, 1, kRThreads, 0, 8LL * n});
}

hipError_t multi_dense(const Launch& l, unsigned nblk, long long lds, const DP* dps, const rkkt_iteration* its,
                       const MultiBlk* blk, hipStream_t s, bool prepare, bool* handled) {
  *handled = true;
  const size_t L = (size_t)lds;
  const unsigned T = (unsigned)l.threads;
  static int cur[8] = {};
  auto go = [&](const void* fn, int slot, auto launch) -> hipError_t {
    if (prepare) return slot >= 0 ? allow_lds(fn, &cur[slot], (int)lds) : hipSuccess;
    launch();
    return hipSuccess;
  };
  switch (l.kernel) {
    case kKSymSum: return go(nullptr, -1, [&] { k_sym_sum_m<<<nblk, T, 0, s>>>(dps, its, blk); });
    case kKStacked:
      switch (l.variant) {
        case 0: return go(nullptr, -1, [&] { k_stacked_product_m<1><<<nblk, T, 0, s>>>(dps, its, blk); });
        case 1: return go(nullptr, -1, [&] { k_stacked_product_m<2><<<nblk, T, 0, s>>>(dps, its, blk); });
        case 2: return go(nullptr, -1, [&] { k_stacked_product_m<4><<<nblk, T, 0, s>>>(dps, its, blk); });
        case 3: return go(nullptr, -1, [&] { k_stacked_product_m<7><<<nblk, T, 0, s>>>(dps, its, blk); });
        default: return go(nullptr, -1, [&] { k_stacked_product_m<kSBMax><<<nblk, T, 0, s>>>(dps, its, blk); });
      }
    case kKCholSmall:
      return go((const void*)k_chol_small_m, 0, [&] { k_chol_small_m<<<nblk, T, L, s>>>(dps, its, blk); });
    case kKCopyChol: return go(nullptr, -1, [&] { k_copy_chol_m<<<nblk, T, 0, s>>>(dps, its, blk); });
    case kKSetInfo: return go(nullptr, -1, [&] { k_set_info_m<<<nblk, T, 0, s>>>(dps, its, blk); });
    case kKCholDiag: return go(nullptr, -1, [&] { k_chol_diag_m<<<nblk, T, 0, s>>>(dps, its, blk, l.jb); });
    case kKCholTrsm: return go(nullptr, -1, [&] { k_chol_trsm_m<<<nblk, T, 0, s>>>(dps, its, blk, l.jb); });
    case kKCholUpdate: return go(nullptr, -1, [&] { k_chol_update_m<<<nblk, T, 0, s>>>(dps, its, blk, l.jb); });
    case kKRSolveBlk:
      return go((const void*)k_reduced_solve_blk_m, 1, [&] { k_reduced_solve_blk_m<<<nblk, T, L, s>>>(dps, its, blk); });
    case kKRSolve:
      if (l.variant == 1)
        return go((const void*)k_reduced_solve_m<true>, 2,
                  [&] { k_reduced_solve_m<true><<<nblk, T, L, s>>>(dps, its, blk); });
      return go((const void*)k_reduced_solve_m<false>, 3,
                [&] { k_reduced_solve_m<false><<<nblk, T, L, s>>>(dps, its, blk); });
    default:
      *handled = false;
      return hipSuccess;
  }
}

}  // namespace rkkt
