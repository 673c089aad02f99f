// Batched sparse LU refactorisation of G_x, the local reduction and the
// single-column solves of the step (paper, parallel KKT solver section: the
// scenario blocks of G_x share one pattern, so their LU factorisations are
// batched; the reduced matrix follows from the three-step product with the
// columns of V = I taken in batches).
//
// Factor layout.  G_x of every scenario is refactorised on one filled pattern
// (fixed symmetric fill-reducing order, static diagonal pivots).  The stored
// factor is L (unit lower), 1/u_ii, and the strict upper part of U with each
// column j scaled by 1/u_jj.  With that scaling every triangular solve is a
// unit-diagonal sweep plus one elementwise scaling:
//   U x = y     : w = (I + U~)^-1 y, x = w / diag(U)
//   U^T z = b   : z = (I + U~^T)^-1 (b / diag(U))
//
// Level-sliced sweeps.  Rows are grouped in levels of the elimination order
// (rows of one level do not depend on each other).  Phase q starts when the
// rows of level q are final; every row that depends on them subtracts those
// contributions.  A phase's work is split over S slots ahead of time (longest
// row first, to the least loaded slot), so the length of the dependency chain
// is the number of phases plus the largest per-slot share of each phase,
// rather than the sum over levels of the longest row.
//
// The refactorisation is the up-looking elimination taken the same way: in
// phase q every entry l_ik with k in level q is divided by u_kk and row k's U
// part is subtracted from row i at precomputed positions.
#include "device.h"

namespace rkkt {

namespace {

constexpr int kRT = kRedThreads;  // reduction workgroup and global-mode scenario group
constexpr int kGT = 256;          // LDS-mode refactor / step workgroup (up to 4 scenarios)

__device__ inline void raise_status(const DP& d, int code, int k) {
  if (atomicCAS(d.status, 0, code) == 0) d.status[1] = k;
}

// dst[idx[e]] = src[e] for e = start, start + stride, ... < n, with
// kStageBatch loads in flight per thread
template <typename T>
__device__ __forceinline__ void scatter_overlapped(T* dst, const int* __restrict__ idx,
                                                   const T* __restrict__ src, int n, int start,
                                                   int stride) {
  for (int e0 = start; e0 < n; e0 += kStageBatch * stride) {
    int id[kStageBatch];
    T v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int e = e0 + u * stride;
      id[u] = e < n ? idx[e] : -1;
      v[u] = e < n ? src[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (id[u] >= 0) dst[id[u]] = v[u];
  }
}

// factor values of scenario k, followed by its 1/u_ii
__device__ __forceinline__ double* lu_of(const DP& d, int k) { return d.LU + (long long)k * d.lu_stride; }

__host__ __device__ __forceinline__ LdsSizes sizes_of(const DP& d) {
  LdsSizes z;
  z.nx = d.nx; z.nu = d.nu; z.nz = d.nz; z.nnz_f = d.nnz_f; z.nnz_k = d.nnz_k;
  z.nnz_gu = d.nnz_gu; z.nnz_l = d.n_sent; z.nlu = d.nlev_up; z.nph_u = d.nph_u;
  z.nph_d = d.nph_d; z.n_upd = d.n_upd; z.w = d.col_tile; z.variant = d.variant; z.spw = d.spw;
  z.nph_ru = d.nph_ru; z.nph_rd = d.nph_rd;
  z.upd_lds = d.upd_lds;
  z.nnz_h = d.nnz_h; z.m = d.m;
  z.chain_t = d.chain_t;
  return z;
}

// schedule entry: four fields, 16-bit packed (LDS copies) or plain int4
struct Ent {
  int a, b, c, d;
};

template <bool kPacked>
__device__ __forceinline__ Ent ent_at(const void* base, int e) {
  if constexpr (kPacked) {
    const uint2 v = static_cast<const uint2*>(base)[e];
    return Ent{(int)(v.x & 0xffffu), (int)(v.x >> 16), (int)(v.y & 0xffffu), (int)(v.y >> 16)};
  } else {
    const int4 v = static_cast<const int4*>(base)[e];
    return Ent{v.x, v.y, v.z, v.w};
  }
}

// One level-sliced unit-diagonal sweep X <- (I + N)^-1 X, N the strict part
// named by the schedule, with values lu[pos] (kTrans: lu[tpos], the mirrored
// entry).  X is row-major with leading dimension ld; this thread owns column
// c and slot `slot` of S.  Every phase ends with sync().
//
// Software pipelining: the schedule entries of the next phase and their
// factor values do not depend on X, so they are loaded into registers (up to
// kPre per thread) while the current phase works; a phase's critical path is
// then the X loads, the multiply-adds and the X stores.  Each dependent row
// is updated in place, X[dest] = ((X[dest] - v0 x0) - v1 x1) ..., in the
// fixed order of the schedule.
constexpr int kPre = 4;

struct PhaseRegs {
  int e0, n;
  int dst[kPre], src[kPre];
  double v[kPre];
};

template <bool kPacked, bool kTrans>
__device__ __forceinline__ void load_phase(PhaseRegs& r, const int* __restrict__ ptr, const void* ent,
                                           const double* __restrict__ lu, int q, int nphase, int S,
                                           int slot, bool act) {
  r.n = 0;
  r.e0 = 0;
  if (!act || q >= nphase) return;
  r.e0 = ptr[q * S + slot];
  r.n = ptr[q * S + slot + 1] - r.e0;
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    if (u < r.n) {
      const Ent t = ent_at<kPacked>(ent, r.e0 + u);
      r.dst[u] = t.a;
      r.src[u] = t.b;
      r.v[u] = lu[kTrans ? t.d : t.c];
    } else {
      r.dst[u] = -1;
      r.src[u] = 0;
      r.v[u] = 0.0;
    }
  }
}

template <bool kPacked, bool kTrans, typename Sync>
__device__ __forceinline__ void sweep(const int* __restrict__ ptr, const void* ent, int nphase, int S,
                                      int slot, bool act, const double* __restrict__ lu, double* X,
                                      int ld, int c, Sync sync) {
  PhaseRegs cur;
  load_phase<kPacked, kTrans>(cur, ptr, ent, lu, 0, nphase, S, slot, act);
  for (int q = 0; q < nphase; ++q) {
    double xs[kPre], xd[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      xs[u] = u < cur.n ? X[(long long)cur.src[u] * ld + c] : 0.0;
      xd[u] = u < cur.n ? X[(long long)cur.dst[u] * ld + c] : 0.0;
    }
    PhaseRegs nxt;
    load_phase<kPacked, kTrans>(nxt, ptr, ent, lu, q + 1, nphase, S, slot, act);
    if (cur.n > 0) {
      double acc = xd[0];
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        if (u < cur.n) {
          acc = fma(-cur.v[u], xs[u], acc);
          const bool last = u + 1 == kPre || u + 1 >= cur.n || cur.dst[u + 1] != cur.dst[u];
          if (last) {
            X[(long long)cur.dst[u] * ld + c] = acc;
            if (u + 1 < kPre) acc = xd[u + 1];
          }
        }
      }
      // entries beyond the registered ones (long tasks), one at a time
      for (int e = cur.e0 + kPre; e < cur.e0 + cur.n; ++e) {
        const Ent t = ent_at<kPacked>(ent, e);
        double* xdp = X + (long long)t.a * ld + c;
        *xdp = fma(-lu[kTrans ? t.d : t.c], X[(long long)t.b * ld + c], *xdp);
      }
    }
    sync();
    cur = nxt;
  }
}

// One sweep for a single right-hand side by one wavefront in LDS (lane =
// slot of kGroupLds), fewest instructions per phase: a phase whose slots hold
// at most one entry each (most phases of these schedules) is one guarded
// multiply-add per lane; longer slots run their entries in order.  Each phase
// issues its own operand reads (from the entry already in registers) together
// with the reads of the next phase's first entry and slot maximum and of the
// slot extent two phases ahead, so the schedule reads no longer form a chain
// of round trips in front of the update; a lane without an entry reads
// through the schedule's first entry and stores nothing.  The wavefront's LDS operations complete in issue order,
// so a phase's reads see the previous phase's stores.
template <bool kTrans, typename Sync>
__device__ __forceinline__ void sweep_w(const int* ptr, const uint2* ent, const int* phmax, int nphase,
                                        int slot, const double* lu, double* X, Sync sync) {
  auto pos = [](uint2 v) { return (int)(kTrans ? v.y >> 16 : v.y & 0xffffu); };
  auto dst = [](uint2 v) { return (int)(v.x & 0xffffu); };
  auto src = [](uint2 v) { return (int)(v.x >> 16); };
  // phase q: extent (e0, n), first entry t, slot maximum m; phase q + 1: the
  // extent's ends (e1, b1) as read
  int e0 = 0, n = 0, m = 0, e1 = 0, b1 = 0;
  uint2 t = make_uint2(0u, 0u);
  if (nphase > 0) {
    e0 = ptr[slot];
    n = ptr[slot + 1] - e0;
    t = ent[n > 0 ? e0 : 0];
    m = phmax[0];
    // reads past the last phase take the last phase's (valid) data, unused
    const int q1 = min(1, nphase - 1);
    e1 = ptr[q1 * kGroupLds + slot];
    b1 = ptr[q1 * kGroupLds + slot + 1];
  }
  for (int q = 0; q < nphase; ++q) {
    const int mq = __builtin_amdgcn_readfirstlane(m);
    const double a = lu[pos(t)], xs = X[src(t)], xd = X[dst(t)];
    const int n1 = b1 - e1, q1 = min(q + 1, nphase - 1), q2 = min(q + 2, nphase - 1);
    const uint2 t1 = ent[n1 > 0 ? e1 : 0];
    const int m1 = phmax[q1];
    const int e2 = ptr[q2 * kGroupLds + slot], b2 = ptr[q2 * kGroupLds + slot + 1];
    if (n > 0) {
      if (mq <= 1) {
        X[dst(t)] = fma(-a, xs, xd);
      } else {
        int cur = dst(t);
        double acc = fma(-a, xs, xd);
        for (int u = 1; u < n; ++u) {
          const uint2 v = ent[e0 + u];
          if (dst(v) != cur) {
            X[cur] = acc;
            cur = dst(v);
            acc = X[cur];
          }
          acc = fma(-lu[pos(v)], X[src(v)], acc);
        }
        X[cur] = acc;
      }
    }
    sync();
    e0 = e1;
    n = n1;
    t = t1;
    m = m1;
    e1 = e2;
    b1 = b2;
  }
}

// ------------------------------------------------------------------ chain
// The chain rows c0 .. nx - 1 (each alone in its level in both directions)
// are solved sequentially in registers instead of one barrier-separated
// phase per row.  Coefficient of (chain row a, chain row b): lu[pos(a, b)];
// the transposed solves read lu[pos(b, a)].

// Positions of the chain coefficients of row a = lane: pos(a, b), or pos(b, a)
// for the transposed solves; -1 where there is none and past the chain.
// Loaded ahead of the solve, so their global round trip overlaps other work.
struct ChainPos {
  int p[kChainMax];
};

template <bool kTrans>
__device__ __forceinline__ ChainPos chain_positions(const DP& d, int lane) {
  ChainPos c;
  const int t = d.chain_t;
  const int* __restrict__ P = d.chain_pos;
  const bool own = lane < t;
#pragma unroll
  for (int b = 0; b < kChainMax; ++b) c.p[b] = own && b < t ? (kTrans ? P[b * t + lane] : P[lane * t + b]) : -1;
  return c;
}

// x_b from lane b of the row for every b < t in order (up) or reverse order
// (down), rows a > b (up) or a < b (down) subtract coef[b] x_b
template <bool kUp, int... B>
__device__ __forceinline__ double chain_row(double x, const double (&coef)[kChainMax], int lane, int t,
                                            std::integer_sequence<int, B...>) {
  auto step = [&](auto bc) {
    constexpr int b = kUp ? decltype(bc)::value : 15 - decltype(bc)::value;
    if (b < t) {
      const double xb = row_bcast<b>(x);
      if (kUp ? lane > b : lane < b) x = fma(-coef[b], xb, x);
    }
  };
  (step(std::integral_constant<int, B>{}), ...);
  return x;
}

// One column, lanes 0 .. t-1 of the calling wavefront hold chain rows a;
// x_b is broadcast with readlane.  Up: b increasing, rows a > b update;
// down: b decreasing, rows a < b update.
// (kDpp: chains of up to 16 rows broadcast with DPP instead of readlane)
template <bool kUp, bool kDpp>
__device__ __forceinline__ void chain_solve1(const DP& d, const double* lu, const ChainPos& cp, double* X,
                                             int lane) {
  const int t = d.chain_t, c0 = d.chain_c0;
  const bool own = lane < t;
  double x = own ? X[c0 + lane] : 0.0;
  double coef[kChainMax];
#pragma unroll
  for (int b = 0; b < kChainMax; ++b) coef[b] = cp.p[b] >= 0 ? lu[cp.p[b]] : 0.0;
  if (kDpp && t <= 16) {
    x = chain_row<kUp>(x, coef, lane, t, std::make_integer_sequence<int, 16>{});
  } else if (kUp) {
#pragma unroll
    for (int b = 0; b < kChainMax; ++b)
      if (b < t) {
        const double xb = readlane_d(x, b);
        if (lane > b) x = fma(-coef[b], xb, x);
      }
  } else {
#pragma unroll
    for (int b = kChainMax - 1; b >= 0; --b)
      if (b < t) {
        const double xb = readlane_d(x, b);
        if (lane < b) x = fma(-coef[b], xb, x);
      }
  }
  if (own) X[c0 + lane] = x;
}

// Many columns: the calling thread solves its own column c of X (leading
// dimension ld) over the chain rows.  cv[a t + b] holds the chain block's
// values (zero where the pattern has no entry), staged in LDS once per
// workgroup, so every coefficient is one broadcast read.
template <bool kUp, bool kTrans>
__device__ __forceinline__ void chain_solveW(const DP& d, const double* cv, double* X, int ld, int c) {
  const int t = d.chain_t, c0 = d.chain_c0;
  double x[kChainMax];
#pragma unroll
  for (int a = 0; a < kChainMax; ++a) x[a] = a < t ? X[(long long)(c0 + a) * ld + c] : 0.0;
  // column order: once x_b is final, every later row subtracts its term; the
  // updates of one step are independent, and each row still subtracts its
  // terms in the order of b
  if (kUp) {
#pragma unroll
    for (int b = 0; b < kChainMax - 1; ++b)
      if (b + 1 < t) {
#pragma unroll
        for (int a = b + 1; a < kChainMax; ++a)
          if (a < t) x[a] = fma(-(kTrans ? cv[b * t + a] : cv[a * t + b]), x[b], x[a]);
      }
  } else {
#pragma unroll
    for (int b = kChainMax - 1; b >= 1; --b)
      if (b < t) {
#pragma unroll
        for (int a = 0; a < b; ++a) x[a] = fma(-(kTrans ? cv[b * t + a] : cv[a * t + b]), x[b], x[a]);
      }
  }
#pragma unroll
  for (int a = 0; a < kChainMax; ++a)
    if (a < t) X[(long long)(c0 + a) * ld + c] = x[a];
}

// Many columns, all wavefronts: wavefront w takes columns 4 w .. 4 w + 3 of
// X, lanes 0..31 holding the chain rows of columns 4 w and 4 w + 2, lanes
// 32..63 those of 4 w + 1 and 4 w + 3; x_b is broadcast with readlane.  The up solve
// and then the down solve, each row subtracting its terms in the same order
// as chain_solveW (so the results are the same).  64 columns = 16
// wavefronts.
// f(integral_constant<int, B>) for B in order
template <typename F, int... B>
__device__ __forceinline__ void for_each_const(F&& f, std::integer_sequence<int, B...>) {
  (f(std::integral_constant<int, B>{}), ...);
}

template <bool kTrans>
__device__ __forceinline__ void chain_solveR(const DP& d, const double* cv, double* X, int ld, int wv) {
  const int t = d.chain_t, c0 = d.chain_c0;
  const int lane = threadIdx.x & 63, a = lane & 31, half = lane >> 5;
  const bool own = a < t;
  // both column pairs of the wavefront at once (independent chains)
  const int col0 = 4 * wv + half, col1 = col0 + 2;
  double x = own ? X[(long long)(c0 + a) * ld + col0] : 0.0;
  double y = own ? X[(long long)(c0 + a) * ld + col1] : 0.0;
  if (t <= 16) {
    // rows in lanes 0..15 (and 32..47 for the other column of the pair):
    // x_b is lane b of each row of 16 lanes, a DPP broadcast
    auto up = [&](auto bc) {
      constexpr int b = decltype(bc)::value;
      if (b < t) {
        const double cf = own ? (kTrans ? cv[b * t + a] : cv[a * t + b]) : 0.0;
        const double xb = row_bcast<b>(x), yb = row_bcast<b>(y);
        if (a > b) {
          x = fma(-cf, xb, x);
          y = fma(-cf, yb, y);
        }
      }
    };
    auto down = [&](auto bc) {
      constexpr int b = 15 - decltype(bc)::value;
      if (b < t) {
        const double cf = own ? (kTrans ? cv[b * t + a] : cv[a * t + b]) : 0.0;
        const double xb = row_bcast<b>(x), yb = row_bcast<b>(y);
        if (a < b) {
          x = fma(-cf, xb, x);
          y = fma(-cf, yb, y);
        }
      }
    };
    for_each_const(up, std::make_integer_sequence<int, 16>{});
    for_each_const(down, std::make_integer_sequence<int, 16>{});
    if (own) {
      X[(long long)(c0 + a) * ld + col0] = x;
      X[(long long)(c0 + a) * ld + col1] = y;
    }
    return;
  }
#pragma unroll
  for (int b = 0; b < kChainMax; ++b)
    if (b < t) {
      const double cf = own ? (kTrans ? cv[b * t + a] : cv[a * t + b]) : 0.0;
      const double x0 = readlane_d(x, b), x1 = readlane_d(x, 32 + b);
      const double y0 = readlane_d(y, b), y1 = readlane_d(y, 32 + b);
      if (a > b) {
        x = fma(-cf, half ? x1 : x0, x);
        y = fma(-cf, half ? y1 : y0, y);
      }
    }
#pragma unroll
  for (int b = kChainMax - 1; b >= 0; --b)
    if (b < t) {
      const double cf = own ? (kTrans ? cv[b * t + a] : cv[a * t + b]) : 0.0;
      const double x0 = readlane_d(x, b), x1 = readlane_d(x, 32 + b);
      const double y0 = readlane_d(y, b), y1 = readlane_d(y, 32 + b);
      if (a < b) {
        x = fma(-cf, half ? x1 : x0, x);
        y = fma(-cf, half ? y1 : y0, y);
      }
    }
  if (own) {
    X[(long long)(c0 + a) * ld + col0] = x;
    X[(long long)(c0 + a) * ld + col1] = y;
  }
}

// chain block values of one scenario into cv (all threads of the workgroup)
__device__ __forceinline__ void chain_gather(const DP& d, const double* lu, double* cv) {
  const int tt = d.chain_t * d.chain_t;
  for (int e = threadIdx.x; e < tt; e += blockDim.x) {
    const int pp = d.chain_pos[e];
    cv[e] = pp >= 0 ? lu[pp] : 0.0;
  }
}

// Up-looking elimination of the chain block after the phases have applied
// every contribution from rows before the chain: lane a holds chain row a
// (zeros where the filled pattern has no entry; the pattern is closed under
// elimination, so they stay zero); row j's pivot and U part are broadcast
// with readlane.  Same pivot test as the phases.
__device__ __forceinline__ void chain_factor(const DP& d, double* lu, double* invd, const double* rmax,
                                             int k, int lane) {
  const int t = d.chain_t, c0 = d.chain_c0;
  const int* __restrict__ P = d.chain_pos;
  const bool own = lane < t;
  // every position load in flight before the first factor value is read
  int pos[kChainMax];
#pragma unroll
  for (int b = 0; b < kChainMax; ++b) pos[b] = own && b < t ? P[lane * t + b] : -1;
  double row[kChainMax];
#pragma unroll
  for (int b = 0; b < kChainMax; ++b) row[b] = pos[b] >= 0 ? lu[pos[b]] : 0.0;
  auto pivot = [&](int j, double ujj) {
    const double inv = 1.0 / ujj;
    if (lane == j) {
      if (!(fabs(ujj) > 0.0 && fabs(ujj) >= 1e-10 * rmax[c0 + j]) || !isfinite(ujj))
        raise_status(d, RKKT_ERR_SINGULAR_GX, k);
      invd[c0 + j] = inv;
    }
    return inv;
  };
  if (t <= 16) {
    // rows in lanes 0..15: row j's entries reach the other rows as DPP
    // broadcasts of lane j within the row of 16 lanes, and only the columns
    // of the chain are touched
    auto elim = [&](auto jc) {
      constexpr int j = decltype(jc)::value;
      if (j < t) {
        const double inv = pivot(j, row_bcast<j>(row[j]));
        const double l = row[j] * inv;
        const bool upd = own && lane > j;
        if (upd) row[j] = l;
#pragma unroll
        for (int b = j + 1; b < 16; ++b)
          if (b < t) {
            const double ub = row_bcast<j>(row[b]);
            if (upd) row[b] = fma(-l, ub, row[b]);
          }
      }
    };
    for_each_const(elim, std::make_integer_sequence<int, 16>{});
  } else {
#pragma unroll
    for (int j = 0; j < kChainMax; ++j) {
      if (j < t) {
        const double inv = pivot(j, readlane_d(row[j], j));
        const double l = row[j] * inv;
        const bool upd = own && lane > j;
        if (upd) row[j] = l;
#pragma unroll
        for (int b = j + 1; b < kChainMax; ++b)
          if (b < t) {
            const double ub = readlane_d(row[b], j);
            if (upd) row[b] = fma(-l, ub, row[b]);
          }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < kChainMax; ++b)
    if (pos[b] >= 0) lu[pos[b]] = row[b];
}

// ------------------------------------------------------------ refactorisation
// LDS mode: spw scenarios per workgroup, one wavefront each, with the shared
// schedule staged once; global mode: one workgroup of kRT threads per scenario.
template <bool kLDS, int kT, bool kUpdLds>
__device__ __forceinline__ void refactor_body(const DP& d, int bx_, int by_, int gx_) {
  constexpr int G = kLDS ? kGroupLds : kT;
  const int tid = threadIdx.x;
  const int gi = kLDS ? tid / G : 0, gl = kLDS ? tid % G : tid;
  const int k = bx_ * (kLDS ? d.spw : 1) + gi;
  const bool live = gi < (kLDS ? d.spw : 1) && k < d.N;
  const int nx = d.nx, nf = d.nnz_f;
  extern __shared__ double smem[];
  double *lu, *invd, *rmax;
  const int *ptr, *upd, *f_ptr, *f_diag, *f_col;
  const void* ent;
  if (kLDS) {
    double* mine = smem + (long long)gi * (nf + 2 * nx);
    lu = mine;
    invd = lu + nf;
    rmax = invd + nx;
    unsigned* ue = reinterpret_cast<unsigned*>(smem + (long long)d.spw * (nf + 2 * nx));
    int* q = reinterpret_cast<int*>(ue + 2 * d.n_sent);
    int* a_p = q; q += d.nph_u * G + 1;
    int* a_lp = q; q += d.nlev_up + 1;
    int* a_lr = q; q += nx;
    int* a_fd = q; q += nx;
    int* a_fp = q; q += nx + 1;
    upd = kUpdLds ? q : d.upd_dst;
    stage_words(ue, d.blob_fac, d.blob_fac_words, tid, blockDim.x);
    (void)a_lp;
    (void)a_lr;
    ptr = a_p; f_diag = a_fd; f_ptr = a_fp;
    f_col = d.f_col;
    ent = ue;
  } else {
    lu = lu_of(d, k);
    invd = lu + nf;
    rmax = d.rhat1 + (long long)k * nx;
    ptr = d.fa_ptr; ent = d.fa_ent; upd = d.upd_dst;
    f_ptr = d.f_ptr; f_diag = d.f_diag; f_col = d.f_col;
  }
  auto gsync = [] {
    if (kLDS) wave_sync();
    else __syncthreads();
  };
  if (live) {
    const double* gv = d.EV + (long long)k * d.n_ev + d.off_gx;
    for (int e = gl; e < nf; e += G) lu[e] = 0.0;
    if (kLDS)
      for (int i = gl; i < nx; i += G) rmax[i] = 0.0;
    gsync();
    if (kLDS) {
      // the values land in the filled pattern, and the largest |entry| of
      // every row of G_x builds up by LDS atomic maxima on the bits of
      // |value| (non-negative doubles order as their bit patterns)
      for (int e0 = gl; e0 < d.nnz_gx; e0 += kStageBatch * G) {
        int id[kStageBatch], row[kStageBatch];
        double v[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
          const int e = e0 + u * G;
          id[u] = e < d.nnz_gx ? d.gx2f[e] : -1;
          row[u] = e < d.nnz_gx ? d.gx_row[e] : 0;
          v[u] = e < d.nnz_gx ? gv[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u)
          if (id[u] >= 0) {
            lu[id[u]] = v[u];
            atomicMax(reinterpret_cast<unsigned long long*>(rmax + row[u]),
                      (unsigned long long)__double_as_longlong(fabs(v[u])));
          }
      }
    } else {
      scatter_overlapped(lu, d.gx2f, gv, d.nnz_gx, gl, G);
    }
  }
  __syncthreads();
  if (!live) return;
  if (!kLDS) {
    // largest |entry| of every row of G_x (fill positions hold zeros)
    for (int i = gl; i < nx; i += G) {
      double mx = 0.0;
      const int e1 = f_ptr[i + 1];
      for (int e = f_ptr[i]; e < e1; ++e) mx = fmax(mx, fabs(lu[e]));
      rmax[i] = mx;
    }
    gsync();
  }
  for (int q = 0; q < d.nph_u; ++q) {
    {
      const int e1 = ptr[q * G + gl + 1];
      for (int e = ptr[q * G + gl]; e < e1; ++e) {
        const Ent t = ent_at<kLDS>(ent, e);  // (position of l_ik, of u_kk, |U(k)|, first target)
        const double l = lu[t.a] * (1.0 / lu[t.b]);
        lu[t.a] = l;
        const int* dst = upd + t.d;
        const double* src = lu + t.b + 1;
        int j = 0;
        for (; j + 4 <= t.c; j += 4) {
          const int d0 = dst[j], d1 = dst[j + 1], d2 = dst[j + 2], d3 = dst[j + 3];
          const double s0 = src[j], s1 = src[j + 1], s2 = src[j + 2], s3 = src[j + 3];
          const double o0 = lu[d0], o1 = lu[d1], o2 = lu[d2], o3 = lu[d3];
          lu[d0] = fma(-l, s0, o0);
          lu[d1] = fma(-l, s1, o1);
          lu[d2] = fma(-l, s2, o2);
          lu[d3] = fma(-l, s3, o3);
        }
        for (; j < t.c; ++j) lu[dst[j]] = fma(-l, src[j], lu[dst[j]]);
      }
    }
    gsync();
  }
  // the chain block, sequentially in registers (one wavefront)
  if (d.chain_t > 0) {
    if (gl < 64) chain_factor(d, lu, invd, rmax, k, gl);
  }
  // pivots of the rows before the chain: test and reciprocal
  for (int i = gl; i < d.chain_c0; i += G) {
    const double p = lu[f_diag[i]];
    if (!(fabs(p) > 0.0 && fabs(p) >= 1e-10 * rmax[i]) || !isfinite(p)) raise_status(d, RKKT_ERR_SINGULAR_GX, k);
    invd[i] = 1.0 / p;
  }
  gsync();
  // scale the columns of the strict upper part by 1/u_jj
  for (int i = gl; i < nx; i += G) {
    const int e1 = f_ptr[i + 1];
    for (int e = f_diag[i] + 1; e < e1; ++e) lu[e] *= invd[f_col[e]];
  }
  if (kLDS) {
    gsync();
    double* glu = lu_of(d, k);  // factor values and 1/u_ii are contiguous in both places
    for (int e = gl; e < nf + nx; e += G) glu[e] = lu[e];
  }
}

template <bool kLDS, int kT, bool kUpdLds>
__global__ __launch_bounds__(kT) void k_refactor(DP d) {
  refactor_body<kLDS, kT, kUpdLds>(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// ---------------------------------------------------------- local reduction
// One workgroup per (tile of W columns of V = I, scenario): slot = thread / W
// (S = kRT / W slots), column = thread % W.
//   step 1: T = -G_x^-1 G_u V            (L sweep, U sweep, scaling)
//   step 2: L_x = K_xx T + K_xu V, L_u = K_ux T + K_uu V
//   step 3 (adjoint, kVar 1): K_hat_k V = L_u - G_u^T G_x^-T L_x, written to part
//   step 3 (product, kVar 2): Z = [T; I] and K Z written to the stacked panels;
//          the stacked product Z^T (K Z) over all scenarios closes the reduction
template <bool kLDS, int kVar>
__device__ __forceinline__ void reduce_body(const DP& d, int bx_, int by_, int gx_) {
  const int k = by_, tile = bx_;
  const int W = d.col_tile, c0 = tile * W, nx = d.nx, nu = d.nu, nz = d.nz;
  const int S = kRT / W;
  const int tid = threadIdx.x, slot = tid / W, c = tid - slot * W;
  const bool act = slot < S;
  const bool colok = act && c0 + c < nu;
  const int col = c0 + c;
  extern __shared__ double smem[];
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double *lu, *invd, *kv, *guv = nullptr;
  double *T, *Lx = nullptr;
  int ldT = W;
  const int *uptr, *dptr, *k_ptr, *k_usplit, *k_col, *guc_ptr, *guc_row;
  const void *uent, *dent;
  double* cv;  // chain block values
  double* zk = kVar == 2 ? d.Zst + (long long)k * nz * d.nu_pad : nullptr;
  double* kzk = kVar == 2 ? d.KZst + (long long)k * nz * d.nu_pad : nullptr;
  if (kLDS) {
    const LdsSizes z = sizes_of(d);
    double* p = smem;
    double* slu = p; p += d.nnz_f;
    double* sid = p; p += nx;
    double* skv = p; p += d.nnz_k;
    double* sgu = p; p += d.nnz_gu;
    T = p; p += (long long)nx * W;
    if (kVar == 1) { Lx = p; p += (long long)nx * W; }
    unsigned* ue = reinterpret_cast<unsigned*>(smem + reduce_lds_doubles(z));
    unsigned* de = ue + 2 * d.n_sent;
    int* ip = reinterpret_cast<int*>(de + 2 * d.n_sent);
    int* a_up = ip; ip += d.nph_ru * S + 1;
    int* a_dp = ip; ip += d.nph_rd * S + 1;
    int* a_kp = ip; ip += nz + 1;
    int* a_ku = ip; ip += nz;
    int* a_kc = ip; ip += d.nnz_k;
    int* a_gp = ip; ip += nu + 1;
    int* a_gr = ip;
    stage_copy(slu, lu_of(d, k), d.nnz_f + nx, tid, kRT);  // factor values, then 1/u_ii into sid
    stage_copy(skv, d.K + (long long)k * d.nnz_k, d.nnz_k, tid, kRT);
    stage_words(ue, d.blob_red, d.blob_red_words, tid, kRT);
    for (int j = tid; j < d.nnz_gu; j += kRT) sgu[j] = ev[d.off_gu + d.guc_pos[j]];
    uptr = a_up; dptr = a_dp; k_ptr = a_kp; k_usplit = a_ku; k_col = a_kc; guc_ptr = a_gp; guc_row = a_gr;
    lu = slu; invd = sid; kv = skv; guv = sgu;
    uent = ue; dent = de;
    cv = smem + (reduce_lds_bytes(z) / 8 - (long long)d.chain_t * d.chain_t);
  } else {
    cv = smem;
    lu = lu_of(d, k);
    invd = lu + d.nnz_f;
    kv = d.K + (long long)k * d.nnz_k;
    if (kVar == 2) {
      T = zk + c0;  // solved in place in the stacked panel
      ldT = d.nu_pad;
    } else {
      T = d.panel + ((long long)k * gx_ + tile) * 2LL * nx * W;
      Lx = T + (long long)nx * W;
    }
    uptr = d.ru_ptr; dptr = d.rd_ptr; uent = d.ru_ent; dent = d.rd_ent;
    k_ptr = d.k_ptr; k_usplit = d.k_usplit; k_col = d.k_col;
    guc_ptr = d.guc_ptr; guc_row = d.guc_row;
  }
  auto bsync = [] { __syncthreads(); };
  auto gu_val = [&](int j) -> double { return kLDS ? guv[j] : ev[d.off_gu + d.guc_pos[j]]; };
  auto k_ucol = [&](int r, int cc) -> double {
    const int e1 = k_ptr[r + 1];
    for (int e = k_usplit[r]; e < e1; ++e)
      if (k_col[e] == cc) return kv[e];
    return 0.0;
  };

  // right-hand side -G_u[:, c0 + c]
  if (colok)
    for (int i = slot; i < nx; i += S) T[(long long)i * ldT + c] = 0.0;
  __syncthreads();
  if (colok)
    for (int j = guc_ptr[col] + slot; j < guc_ptr[col + 1]; j += S)
      T[(long long)guc_row[j] * ldT + c] = -gu_val(j);
  chain_gather(d, lu, cv);
  __syncthreads();
  // step 1
  const bool chain_lane = slot == 0 && (kLDS || colok);
  sweep<kLDS, false>(uptr, uent, d.nph_ru, S, slot, colok, lu, T, ldT, c, bsync);
  if (d.chain_t > 0) {
    if (chain_lane) chain_solveW<true, false>(d, cv, T, ldT, c);
    __syncthreads();
    if (chain_lane) chain_solveW<false, false>(d, cv, T, ldT, c);
    __syncthreads();
  }
  sweep<kLDS, false>(dptr, dent, d.nph_rd, S, slot, colok, lu, T, ldT, c, bsync);
  if (colok)
    for (int i = slot; i < nx; i += S) T[(long long)i * ldT + c] *= invd[i];
  __syncthreads();
  if (kVar == 2) {
    if (!colok) return;
    if (kLDS)
      for (int i = slot; i < nx; i += S) zk[(long long)i * d.nu_pad + col] = T[i * W + c];
    for (int r = slot; r < nz; r += S) {
      double acc = k_ucol(r, nx + col);
      const int e1 = k_usplit[r];
      for (int e = k_ptr[r]; e < e1; ++e) acc = fma(kv[e], T[(long long)k_col[e] * ldT + c], acc);
      kzk[(long long)r * d.nu_pad + col] = acc;
    }
    return;
  }
  // step 2 (adjoint): L_x, prescaled by 1/u_ii for the U^T sweep; L_u into part
  double* out = d.part + (long long)k * nu * nu;
  if (colok)
    for (int r = slot; r < nz; r += S) {
      double acc = k_ucol(r, nx + col);
      const int e1 = k_usplit[r];
      for (int e = k_ptr[r]; e < e1; ++e) acc = fma(kv[e], T[(long long)k_col[e] * W + c], acc);
      if (r < nx) Lx[(long long)r * W + c] = acc * invd[r];
      else out[(long long)(r - nx) * nu + col] = acc;
    }
  __syncthreads();
  // step 3: U^T sweep, L^T sweep, then L_u - G_u^T (G_x^-T L_x)
  sweep<kLDS, true>(uptr, uent, d.nph_ru, S, slot, colok, lu, Lx, W, c, bsync);
  if (d.chain_t > 0) {
    if (chain_lane) chain_solveW<true, true>(d, cv, Lx, W, c);
    __syncthreads();
    if (chain_lane) chain_solveW<false, true>(d, cv, Lx, W, c);
    __syncthreads();
  }
  sweep<kLDS, true>(dptr, dent, d.nph_rd, S, slot, colok, lu, Lx, W, c, bsync);
  if (colok)
    for (int ru = slot; ru < nu; ru += S) {
      double acc = out[(long long)ru * nu + col];
      const int j1 = guc_ptr[ru + 1];
      for (int j = guc_ptr[ru]; j < j1; ++j) acc = fma(-gu_val(j), Lx[(long long)guc_row[j] * W + c], acc);
      out[(long long)ru * nu + col] = acc;
    }
}

template <bool kLDS, int kVar>
__global__ __launch_bounds__(kRT) void k_reduce(DP d) {
  reduce_body<kLDS, kVar>(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// ------------------------------------- local reduction with 64-column tiles
// One slot per wavefront (lane = column, S = 16 slots): the schedule entries,
// the K pattern and the factor values a wavefront reads are the same for all
// of its lanes, so the schedule and the pattern come through scalar loads
// (wave-uniform indices) and the factor values as LDS broadcasts; only the
// panel arithmetic runs on the vector unit.  Entries of a phase are taken
// four at a time with all their loads issued first.
constexpr int kW64 = 64, kS64 = kRT / kW64;

template <bool kTrans, typename Sync>
__device__ __forceinline__ void sweep64(const int* __restrict__ ptr, const int4* __restrict__ ent,
                                        int nphase, int wv, const double* __restrict__ lu, double* X,
                                        int ld, int c, Sync sync) {
  // Software pipeline over phases with vector loads, which have a wait
  // counter of their own, so the phase's LDS waits never wait for them:
  // phase bounds three phases ahead (lanes 0 and 1), entries two phases
  // ahead and factor values one phase ahead (lane u holds entry u).
  const int lane = threadIdx.x & 63;
  auto bounds = [&](int q) -> int {
    return q < nphase && lane < 2 ? ptr[q * kS64 + wv + lane] : 0;
  };
  auto first = [](int bq) { return __builtin_amdgcn_readlane(bq, 0); };
  auto count = [](int bq) { return __builtin_amdgcn_readlane(bq, 1) - __builtin_amdgcn_readlane(bq, 0); };
  auto entries = [&](int bq) -> int4 {
    const int b = first(bq), n = count(bq);
    return lane < n ? ent[b + lane] : make_int4(-1, 0, 0, 0);
  };
  auto values = [&](int4 ev) -> double { return ev.x >= 0 ? lu[kTrans ? ev.w : ev.z] : 0.0; };
  int bq0 = bounds(0), bq1 = bounds(1), bq2 = bounds(2);
  int4 ev0 = entries(bq0), ev1 = entries(bq1);
  double lv0 = values(ev0);
  for (int q = 0; q < nphase; ++q) {
    const double lv1 = values(ev1);
    const int4 ev2 = entries(bq2);
    const int bq3 = bounds(q + 3);
    const int b0 = first(bq0), n = count(bq0);
    int cur = -1;
    double acc = 0.0;
    const int m = min(n, 64);
    for (int u = 0; u < m; ++u) {
      const int dst = __builtin_amdgcn_readlane(ev0.x, u), src = __builtin_amdgcn_readlane(ev0.y, u);
      const double v = readlane_d(lv0, u);
      const double x = X[src * ld + c];
      if (dst != cur) {
        if (cur >= 0) X[cur * ld + c] = acc;
        cur = dst;
        acc = X[cur * ld + c];
      }
      acc = fma(-v, x, acc);
    }
    // entries past the 64 held in lanes, one at a time
    for (int e = b0 + 64; e < b0 + n; ++e) {
      const int4 t = ent[e];
      const double x = X[t.y * ld + c];
      if (t.x != cur) {
        if (cur >= 0) X[cur * ld + c] = acc;
        cur = t.x;
        acc = X[cur * ld + c];
      }
      acc = fma(-lu[kTrans ? t.w : t.z], x, acc);
    }
    if (cur >= 0) X[cur * ld + c] = acc;
    sync();
    bq0 = bq1;
    bq1 = bq2;
    bq2 = bq3;
    ev0 = ev1;
    ev1 = ev2;
    lv0 = lv1;
  }
}

// The same sweep with the panel X and the factor in global memory (panels
// too large for LDS): each load is a round trip to L2 or HBM, so the
// entries of a phase are taken in batches of kGB whose panel loads (the
// source row's value and the destination row's current value) are all
// issued before the batch's multiply-adds.  Within a phase the source rows
// are final and each destination row belongs to one slot as one contiguous
// group, so a prefetched destination value is current whenever its group
// starts in the batch (a group that continues from the previous batch keeps
// its running sum in a register).  Entries are held in lanes in chunks of
// 64, the next chunk and its factor values loaded while the current one
// runs.  Every destination subtracts its terms in schedule order, as in
// sweep64.
constexpr int kGB = 16;

template <bool kTrans, typename Sync>
__device__ __forceinline__ void sweep64g(const int* __restrict__ ptr, const int4* __restrict__ ent,
                                         int nphase, int wv, const double* __restrict__ lu, double* X,
                                         int ld, int c, Sync sync) {
  const int lane = threadIdx.x & 63;
  auto chunk = [&](int e, int b1) -> int4 { return e + lane < b1 ? ent[e + lane] : make_int4(-1, 0, 0, 0); };
  auto values = [&](int4 ev) -> double { return ev.x >= 0 ? lu[kTrans ? ev.w : ev.z] : 0.0; };
  int bq = lane < 2 ? ptr[wv + lane] : 0;
  for (int q = 0; q < nphase; ++q) {
    const int b0 = __builtin_amdgcn_readlane(bq, 0), b1 = __builtin_amdgcn_readlane(bq, 1);
    bq = q + 1 < nphase && lane < 2 ? ptr[(q + 1) * kS64 + wv + lane] : 0;
    int4 ev = chunk(b0, b1);
    double lv = values(ev);
    int cur = -1;
    double acc = 0.0;
    for (int e0 = b0; e0 < b1; e0 += 64) {
      const int m = min(64, b1 - e0);
      const int4 evn = chunk(e0 + 64, b1);
      const double lvn = values(evn);
      for (int u0 = 0; u0 < m; u0 += kGB) {
        double xs[kGB], xd[kGB];
#pragma unroll
        for (int j = 0; j < kGB; ++j) {
          if (u0 + j < m) {
            const int dst = __builtin_amdgcn_readlane(ev.x, u0 + j);
            const int src = __builtin_amdgcn_readlane(ev.y, u0 + j);
            xs[j] = X[(long long)src * ld + c];
            xd[j] = X[(long long)dst * ld + c];
          }
        }
#pragma unroll
        for (int j = 0; j < kGB; ++j) {
          if (u0 + j < m) {
            const int dst = __builtin_amdgcn_readlane(ev.x, u0 + j);
            const double v = readlane_d(lv, u0 + j);
            if (dst != cur) {
              if (cur >= 0) X[(long long)cur * ld + c] = acc;
              cur = dst;
              acc = xd[j];
            }
            acc = fma(-v, xs[j], acc);
          }
        }
      }
      ev = evn;
      lv = lvn;
    }
    if (cur >= 0) X[(long long)cur * ld + c] = acc;
    sync();
  }
}

template <bool kTrans, bool kLDS, typename Sync>
__device__ __forceinline__ void sweep64_any(const int* __restrict__ ptr, const int4* __restrict__ ent,
                                            int nphase, int wv, const double* __restrict__ lu, double* X,
                                            int ld, int c, Sync sync) {
  if constexpr (kLDS) sweep64<kTrans>(ptr, ent, nphase, wv, lu, X, ld, c, sync);
  else sweep64g<kTrans>(ptr, ent, nphase, wv, lu, X, ld, c, sync);
}

template <bool kLDS, int kVar>
__device__ __forceinline__ void reduce64_body(const DP& d, int bx_, int by_, int gx_) {
  const int k = by_, tile = bx_;
  const int c0 = tile * kW64, nx = d.nx, nu = d.nu, nz = d.nz;
  const int tid = threadIdx.x, c = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = c0 + c;
  const bool colok = col < nu;
  extern __shared__ double smem[];
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double *lu, *invd, *guv = nullptr;
  const double* kv;
  double *T, *Lx = nullptr;
  int ldT = kW64;
  double* zk = kVar == 2 ? d.Zst + (long long)k * nz * d.nu_pad : nullptr;
  double* kzk = kVar == 2 ? d.KZst + (long long)k * nz * d.nu_pad : nullptr;
  const int* k_ptr = d.k_ptr;
  const int* k_usplit = d.k_usplit;
  const int* k_col = d.k_col;
  kv = d.K + (long long)k * d.nnz_k;
  double* cv = smem;  // chain block values (global mode: the only LDS use)
  if (kLDS) {
    double* p = smem;
    double* slu = p; p += d.nnz_f + nx;
    double* skv = p; p += d.nnz_k;
    double* sgu = p; p += d.nnz_gu;
    T = p; p += (long long)nx * kW64;
    if (kVar == 1) { Lx = p; p += (long long)nx * kW64; }
    int* ip = reinterpret_cast<int*>(p);
    int* skp = ip; ip += nz + 1;
    int* sku = ip; ip += nz;
    int* skc = ip;
    // Staging: the loads of every array (factor values and 1/u_ii, K values
    // and pattern, the scenario's G_u values) are in flight together before
    // the first LDS store, about two round trips to L2 or HBM in all (the
    // G_u values wait for their positions) instead of one or more per array.
    {
      constexpr int kB = 4;  // elements per thread and array in flight
      const int nlu = d.nnz_f + nx, nk = d.nnz_k, ngu = d.nnz_gu;
      const double* glu = lu_of(d, k);
      const double* gk = d.K + (long long)k * nk;
      const int nmax = max(max(nlu, nk), max(nz + 1, ngu));
      for (int i0 = tid; i0 < nmax; i0 += kB * kRT) {
        double va[kB], vb[kB], vg[kB];
        int ia[kB], ib[kB], ic[kB], ig[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int i = i0 + u * kRT;
          if (i < nlu) va[u] = glu[i];
          if (i < nk) {
            vb[u] = gk[i];
            ic[u] = d.k_col[i];
          }
          if (i <= nz) ia[u] = d.k_ptr[i];
          if (i < nz) ib[u] = d.k_usplit[i];
          if (i < ngu) ig[u] = d.guc_pos[i];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u)
          if (i0 + u * kRT < ngu) vg[u] = ev[d.off_gu + ig[u]];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int i = i0 + u * kRT;
          if (i < nlu) slu[i] = va[u];
          if (i < nk) {
            skv[i] = vb[u];
            skc[i] = ic[u];
          }
          if (i <= nz) skp[i] = ia[u];
          if (i < nz) sku[i] = ib[u];
          if (i < ngu) sgu[i] = vg[u];
        }
      }
    }
    k_ptr = skp;
    k_usplit = sku;
    k_col = skc;
    kv = skv;
    cv = smem + (reduce_lds_bytes(sizes_of(d)) / 8 - (long long)d.chain_t * d.chain_t);
    lu = slu; invd = slu + d.nnz_f; guv = sgu;
  } else {
    lu = lu_of(d, k);
    invd = lu + d.nnz_f;
    if (kVar == 2) {
      T = zk + c0;  // solved in place in the stacked panel
      ldT = d.nu_pad;
    } else {
      T = d.panel + ((long long)k * gx_ + tile) * 2LL * nx * kW64;
      Lx = T + (long long)nx * kW64;
    }
  }
  auto bsync = [] { __syncthreads(); };
  auto gu_val = [&](int j) -> double { return kLDS ? guv[j] : ev[d.off_gu + d.guc_pos[j]]; };
  // right-hand side -G_u[:, c0 + c] (padding columns: zero)
  for (int i = wv; i < nx; i += kS64) T[(long long)i * ldT + c] = 0.0;
  __syncthreads();
  if (colok)
    for (int j = d.guc_ptr[col] + wv; j < d.guc_ptr[col + 1]; j += kS64)
      T[(long long)d.guc_row[j] * ldT + c] = -gu_val(j);
  chain_gather(d, lu, cv);
  __syncthreads();
  // step 1: T = -G_x^-1 G_u V
  const int4* uent = static_cast<const int4*>(d.ru_ent);
  const int4* dent = static_cast<const int4*>(d.rd_ent);
  // every lane sweeps (barriers stay uniform); lanes past n_u work on
  // padding columns inside the panel, which nothing reads
  sweep64_any<false, kLDS>(d.ru_ptr, uent, d.nph_ru, wv, lu, T, ldT, c, bsync);
  if (d.chain_t > 0) {
    chain_solveR<false>(d, cv, T, ldT, wv);
    __syncthreads();
  }
  sweep64_any<false, kLDS>(d.rd_ptr, dent, d.nph_rd, wv, lu, T, ldT, c, bsync);
  if (colok)
    for (int i = wv; i < nx; i += kS64) T[(long long)i * ldT + c] *= invd[i];
  __syncthreads();
  // step 2: rows of K, four rows per wavefront at a time (independent
  // chains).  A row's entries are read lane-parallel (lane u holds entry u,
  // one vector read per array) and broadcast with readlane, so the LDS pipe
  // carries only the panel reads; rows longer than 64 entries take the
  // entry-by-entry path.
  constexpr int kRowsK = 4;
  auto k_rows = [&](int r0, double out4[kRowsK]) {
    int e[kRowsK], eu[kRowsK], e1[kRowsK];
    int len = 0, longest = 0;
#pragma unroll
    for (int j = 0; j < kRowsK; ++j) {
      const int r = r0 + j * kS64;
      e[j] = r < nz ? k_ptr[r] : 0;
      eu[j] = r < nz ? k_usplit[r] : 0;
      e1[j] = r < nz ? k_ptr[r + 1] : 0;
      len = max(len, eu[j] - e[j]);
      longest = max(longest, e1[j] - e[j]);
    }
    if (longest > 64) return false;
    const int lane = threadIdx.x & 63;
    int colv[kRowsK];
    double valv[kRowsK], acc[kRowsK];
#pragma unroll
    for (int j = 0; j < kRowsK; ++j) {
      const bool in = lane < e1[j] - e[j];
      colv[j] = in ? k_col[e[j] + lane] : -1;
      valv[j] = in ? kv[e[j] + lane] : 0.0;
      acc[j] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < kRowsK; ++j)
      for (int m = eu[j] - e[j]; m < e1[j] - e[j]; ++m) {
        const int cm = __builtin_amdgcn_readlane(colv[j], m);
        const double vm = readlane_d(valv[j], m);
        if (cm == nx + col) acc[j] = vm;
      }
    // panel values of kRowsB entries of every row loaded before their
    // multiply-adds (each row still sums its entries in pattern order)
    constexpr int kRowsB = 8;
    for (int m0 = 0; m0 < len; m0 += kRowsB) {
      double tv[kRowsK][kRowsB];
#pragma unroll
      for (int j = 0; j < kRowsK; ++j)
#pragma unroll
        for (int t = 0; t < kRowsB; ++t)
          if (m0 + t < eu[j] - e[j])
            tv[j][t] = T[(long long)__builtin_amdgcn_readlane(colv[j], m0 + t) * ldT + c];
#pragma unroll
      for (int j = 0; j < kRowsK; ++j)
#pragma unroll
        for (int t = 0; t < kRowsB; ++t)
          if (m0 + t < eu[j] - e[j]) acc[j] = fma(readlane_d(valv[j], m0 + t), tv[j][t], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < kRowsK; ++j) out4[j] = acc[j];
    return true;
  };
  auto k_rows_slow = [&](int r0, double out4[kRowsK]) {
    int e[kRowsK], eu[kRowsK], e1[kRowsK];
    int len = 0;
#pragma unroll
    for (int j = 0; j < kRowsK; ++j) {
      const int r = r0 + j * kS64;
      e[j] = r < nz ? k_ptr[r] : 0;
      eu[j] = r < nz ? k_usplit[r] : 0;
      e1[j] = r < nz ? k_ptr[r + 1] : 0;
      len = max(len, eu[j] - e[j]);
    }
    double acc[kRowsK];
#pragma unroll
    for (int j = 0; j < kRowsK; ++j) {
      acc[j] = 0.0;
      for (int q = eu[j]; q < e1[j]; ++q)
        if (k_col[q] == nx + col) acc[j] = kv[q];
    }
    for (int m = 0; m < len; ++m) {
#pragma unroll
      for (int j = 0; j < kRowsK; ++j) {
        const int q = e[j] + m;
        if (q < eu[j]) acc[j] = fma(kv[q], T[(long long)k_col[q] * ldT + c], acc[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < kRowsK; ++j) out4[j] = acc[j];
  };
  // k_rows reads a row's entries across all 64 lanes, so every lane runs it
  // (padding columns of the panel are zero and match no u column) and only
  // the stores are limited to columns < n_u
  if (kVar == 2) {
    if (kLDS && colok)
      for (int i = wv; i < nx; i += kS64) zk[(long long)i * d.nu_pad + col] = T[i * kW64 + c];
    if (kLDS) {
      // (row, 16-column quarter) items over all threads: a row's entries are
      // read once per item and each multiplies 16 panel values; the lanes
      // take the quarter's columns in lane-rotated order, so the panel reads
      // of one instruction spread over the LDS banks.  Each value is
      // K[r][n_x + col] plus the x entries' terms in pattern order.
      const int ln = (tid >> 2) & 15;
      // the terms of row r from entries [e0, e1) into acc (the quarter at
      // column lo), the u-part value K[r][n_x + col] first when `head`
      auto item = [&](int r, int e0, int e1, bool head, int lo, double (&acc)[16]) {
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.0;
        if (head)
          for (int e = k_usplit[r]; e < k_ptr[r + 1]; ++e) {
            const int cu = k_col[e] - nx - c0 - lo;
            const double v = kv[e];
#pragma unroll
            for (int j = 0; j < 16; ++j)
              if (((j + ln) & 15) == cu) acc[j] = v;
          }
        for (int e = e0; e < e1; ++e) {
          const double v = kv[e];
          const double* tr = T + (long long)k_col[e] * kW64 + lo;
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[j] = fma(v, tr[(j + ln) & 15], acc[j]);
        }
      };
      if (d.n_kz > 0) {
        // Items (piece of a K row, 16-column quarter), the longest pieces
        // first, at most kKzItems per thread.  A thread's items stay in
        // registers until every panel read is done; the rows then pass
        // through LDS (the whole workgroup's LDS is dead by then), the pieces
        // of a row added in piece order one round each, and leave as whole
        // 512-byte rows instead of one 8-byte store per value (the 8-byte
        // stores, spread over the row items, measured 3 us slower per launch
        // on the 118-bus grid).
        const int4* items = reinterpret_cast<const int4*>(d.kz_items);
        double res[kKzItems][16];
        int4 pc[kKzItems];
#pragma unroll
        for (int u = 0; u < kKzItems; ++u) {
          const int it = tid + u * kRT;
          pc[u] = it < 4 * d.n_kz ? items[it >> 2] : make_int4(-1, 0, 0, -1);
          if (pc[u].x >= 0) item(pc[u].x, pc[u].y, pc[u].z, pc[u].w == 0, 16 * (tid & 3), res[u]);
        }
        __syncthreads();
        const int rows = (int)(reduce_lds_bytes(sizes_of(d)) / (8 * kW64));
        for (int rb = 0; rb < nz; rb += rows) {
          for (int q = 0; q < d.kz_rounds; ++q) {
#pragma unroll
            for (int u = 0; u < kKzItems; ++u) {
              const int r = pc[u].x - rb, lo = 16 * (tid & 3);
              if (pc[u].w == q && r >= 0 && r < rows) {
                double* srow = smem + (long long)r * kW64 + lo;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                  const int cj = (j + ln) & 15;
                  srow[cj] = q == 0 ? res[u][j] : srow[cj] + res[u][j];
                }
              }
            }
            __syncthreads();
          }
          const int rn = min(rows, nz - rb);
          if (colok)
            for (int r = wv; r < rn; r += kS64) kzk[(long long)(rb + r) * d.nu_pad + col] = smem[r * kW64 + c];
          if (rb + rows < nz) __syncthreads();
        }
        return;
      }
      for (int it = tid; it < nz * 4; it += kRT) {
        const int r = it >> 2, lo = 16 * (it & 3);
        double acc[16];
        item(r, k_ptr[r], k_usplit[r], true, lo, acc);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int cc = c0 + lo + ((j + ln) & 15);
          if (cc < nu) kzk[(long long)r * d.nu_pad + cc] = acc[j];
        }
      }
      return;
    }
    for (int r0 = wv; r0 < nz; r0 += kRowsK * kS64) {
      double v[kRowsK];
      if (!k_rows(r0, v)) k_rows_slow(r0, v);
#pragma unroll
      for (int j = 0; j < kRowsK; ++j)
        if (colok && r0 + j * kS64 < nz) kzk[(long long)(r0 + j * kS64) * d.nu_pad + col] = v[j];
    }
    return;
  }
  // adjoint: L_x (prescaled by 1/u_ii for the U^T sweep), L_u into part
  double* out = d.part + (long long)k * nu * nu;
  for (int r0 = wv; r0 < nz; r0 += kRowsK * kS64) {
    double v[kRowsK];
    if (!k_rows(r0, v)) k_rows_slow(r0, v);
#pragma unroll
    for (int j = 0; j < kRowsK; ++j) {
      const int r = r0 + j * kS64;
      if (r < nx) Lx[(long long)r * kW64 + c] = colok ? v[j] * invd[r] : 0.0;
      else if (r < nz && colok) out[(long long)(r - nx) * nu + col] = v[j];
    }
  }
  __syncthreads();
  sweep64_any<true, kLDS>(d.ru_ptr, uent, d.nph_ru, wv, lu, Lx, kW64, c, bsync);
  if (d.chain_t > 0) {
    chain_solveR<true>(d, cv, Lx, kW64, wv);
    __syncthreads();
  }
  sweep64_any<true, kLDS>(d.rd_ptr, dent, d.nph_rd, wv, lu, Lx, kW64, c, bsync);
  // G_u^T product: the entries of a column of G_u loaded kGB at a time
  // before their multiply-adds (summed in pattern order)
  if (colok)
    for (int ru = wv; ru < nu; ru += kS64) {
      double acc = out[(long long)ru * nu + col];
      const int j1 = d.guc_ptr[ru + 1];
      for (int jb = d.guc_ptr[ru]; jb < j1; jb += kGB) {
        double gv[kGB], lx[kGB];
#pragma unroll
        for (int t = 0; t < kGB; ++t)
          if (jb + t < j1) {
            gv[t] = gu_val(jb + t);
            lx[t] = Lx[(long long)d.guc_row[jb + t] * kW64 + c];
          }
#pragma unroll
        for (int t = 0; t < kGB; ++t)
          if (jb + t < j1) acc = fma(-gv[t], lx[t], acc);
      }
      out[(long long)ru * nu + col] = acc;
    }
}

template <bool kLDS, int kVar>
__global__ __launch_bounds__(kRT) void k_reduce64(DP d) {
  reduce64_body<kLDS, kVar>(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// ------------------------------------------------ single-column solves (step)
// LDS mode: one workgroup of kGT threads per scenario stages everything the
// scenario's step reads (factor and 1/u_ii, K, H and G_u values, the
// residual vectors, the schedules) in one overlapped pass; the elementwise
// work uses all threads on LDS data and the triangular sweeps run on
// wavefront 0 (one slot per lane, wavefront-scope synchronisation).  Global
// mode: one workgroup of kRT threads per scenario on global data, sweeps on
// all threads.
struct StepView {
  const double *lu, *invd, *Kv, *hv, *guv;
  const double *ra, *r3, *r2, *r4, *ss, *pu;  // ra: r1x (rhs) or rhat1 (recovery)
  double *v0, *v1, *v2, *wv;
  const int *uptr, *dptr;
  const void *uent, *dent;
  const int *umax, *dmax;  // LDS mode: largest slot count of each phase
};

template <bool kLDS>
__device__ __forceinline__ StepView step_view(const DP& d, int k, double* smem, const double* ra,
                                              const double* r3, const double* r2, const double* r4,
                                              const double* ss, const double* pu) {
  StepView w;
  const int nx = d.nx, nf = d.nnz_f, m = d.m;
  const double* ev = d.EV + (long long)k * d.n_ev;
  if (kLDS) {
    double* p = smem;
    double* lu = p; p += nf + nx;
    double* kv = p; p += d.nnz_k;
    double* hv = p; p += d.nnz_h;
    double* gu = p; p += d.nnz_gu;
    double* sra = p; p += nx;
    double* sr3 = p; p += nx;
    double* sr2 = p; p += m;
    double* sr4 = p; p += m;
    double* sss = p; p += m;
    w.wv = p; p += m;
    w.v0 = p; p += nx;
    w.v1 = p; p += nx;
    w.v2 = p; p += nx;
    double* spu = p; p += d.nu;
    unsigned* ue = reinterpret_cast<unsigned*>(p);
    unsigned* de = ue + 2 * d.n_sent;
    int* ip = reinterpret_cast<int*>(de + 2 * d.n_sent);
    w.uptr = ip;
    w.dptr = ip + d.nph_u * kGroupLds + 1;
    w.umax = w.dptr + d.nph_d * kGroupLds + 1;
    w.dmax = w.umax + d.nph_u;
    w.uent = ue;
    w.dent = de;
    const int t0 = threadIdx.x, ts = blockDim.x;
    stage_copy(lu, lu_of(d, k), nf + nx, t0, ts);
    stage_copy(kv, d.K + (long long)k * d.nnz_k, d.nnz_k, t0, ts);
    stage_copy(hv, ev + d.off_h, d.nnz_h, t0, ts);
    stage_copy(gu, ev + d.off_gu, d.nnz_gu, t0, ts);
    stage_copy(sra, ra + (long long)k * nx, nx, t0, ts);
    stage_copy(sr3, r3 + (long long)k * nx, nx, t0, ts);
    stage_copy(sr2, r2 + (long long)k * m, m, t0, ts);
    stage_copy(sr4, r4 + (long long)k * m, m, t0, ts);
    stage_copy(sss, ss + (long long)k * m, m, t0, ts);
    if (pu) stage_copy(spu, pu, d.nu, t0, ts);
    stage_words(ue, d.blob_stp, d.blob_stp_words, t0, ts);
    w.lu = lu; w.invd = lu + nf; w.Kv = kv; w.hv = hv; w.guv = gu;
    w.ra = sra; w.r3 = sr3; w.r2 = sr2; w.r4 = sr4; w.ss = sss; w.pu = spu;
  } else {
    w.lu = lu_of(d, k);
    w.invd = w.lu + nf;
    w.Kv = d.K + (long long)k * d.nnz_k;
    w.hv = ev + d.off_h;
    w.guv = ev + d.off_gu;
    w.ra = ra + (long long)k * nx;
    w.r3 = r3 + (long long)k * nx;
    w.r2 = r2 + (long long)k * m;
    w.r4 = r4 + (long long)k * m;
    w.ss = ss + (long long)k * m;
    w.pu = pu;
    w.v0 = d.panel + (long long)k * 2 * nx;
    w.v1 = w.v0 + nx;
    w.v2 = d.rhat1 + (long long)k * nx;
    w.wv = d.wbuf + (long long)k * m;
    w.uptr = d.su_ptr; w.dptr = d.sd_ptr; w.uent = d.su_ent; w.dent = d.sd_ent;
    w.umax = w.dmax = nullptr;
  }
  __syncthreads();
  return w;
}

// X <- G_x^-1 X (internal order) by the sweep group (G threads, slot gl);
// cp: chain_positions<false> of slot gl
template <bool kLDS, typename Sync>
__device__ __forceinline__ void solve_fwd(const DP& d, const StepView& w, double* X, int gl, Sync sync,
                                          const ChainPos& cp) {
  constexpr int G = kLDS ? kGroupLds : kRT;
  if (kLDS) sweep_w<false>(w.uptr, static_cast<const uint2*>(w.uent), w.umax, d.nph_u, gl, w.lu, X, sync);
  else sweep<kLDS, false>(w.uptr, w.uent, d.nph_u, G, gl, true, w.lu, X, 1, 0, sync);
  if (d.chain_t > 0) {
    if (gl < 64) chain_solve1<true, kLDS>(d, w.lu, cp, X, gl);
    sync();
    if (gl < 64) chain_solve1<false, kLDS>(d, w.lu, cp, X, gl);
    sync();
  }
  if (kLDS) sweep_w<false>(w.dptr, static_cast<const uint2*>(w.dent), w.dmax, d.nph_d, gl, w.lu, X, sync);
  else sweep<kLDS, false>(w.dptr, w.dent, d.nph_d, G, gl, true, w.lu, X, 1, 0, sync);
  for (int i = gl; i < d.nx; i += G) X[i] *= w.invd[i];
  sync();
}

template <bool kLDS, typename Sync>
__device__ __forceinline__ void solve_fwd(const DP& d, const StepView& w, double* X, int gl, Sync sync) {
  solve_fwd<kLDS>(d, w, X, gl, sync, chain_positions<false>(d, gl));
}

// X <- G_x^-T X for X already scaled by 1/u_ii; cp: chain_positions<true>
template <bool kLDS, typename Sync>
__device__ __forceinline__ void solve_adj_scaled(const DP& d, const StepView& w, double* X, int gl, Sync sync,
                                                 const ChainPos& cp) {
  constexpr int G = kLDS ? kGroupLds : kRT;
  if (kLDS) sweep_w<true>(w.uptr, static_cast<const uint2*>(w.uent), w.umax, d.nph_u, gl, w.lu, X, sync);
  else sweep<kLDS, true>(w.uptr, w.uent, d.nph_u, G, gl, true, w.lu, X, 1, 0, sync);
  if (d.chain_t > 0) {
    if (gl < 64) chain_solve1<true, kLDS>(d, w.lu, cp, X, gl);
    sync();
    if (gl < 64) chain_solve1<false, kLDS>(d, w.lu, cp, X, gl);
    sync();
  }
  if (kLDS) sweep_w<true>(w.dptr, static_cast<const uint2*>(w.dent), w.dmax, d.nph_d, gl, w.lu, X, sync);
  else sweep<kLDS, true>(w.dptr, w.dent, d.nph_d, G, gl, true, w.lu, X, 1, 0, sync);
  sync();
}

template <bool kLDS, typename Sync>
__device__ __forceinline__ void solve_adj_scaled(const DP& d, const StepView& w, double* X, int gl, Sync sync) {
  solve_adj_scaled<kLDS>(d, w, X, gl, sync, chain_positions<true>(d, gl));
}

// runs a sweep-group solve: wavefront 0 in LDS mode, every thread otherwise
template <bool kLDS, typename F>
__device__ __forceinline__ void in_sweep_group(F f) {
  if (kLDS) {
    if ((threadIdx.x >> 6) == 0) f(threadIdx.x & 63, [] { wave_sync(); });
  } else {
    f(threadIdx.x, [] { __syncthreads(); });
  }
  __syncthreads();
}

// Reduced right-hand side contributions of one scenario (eq. "kkt:reduced"):
//   rhat1 = r1x + H_x^T (Sigma_s r4 - r2),  q = G_x^-1 r3,
//   a = G_x^-T (rhat1 - K_xx q),
//   rpart = -H_u^T (Sigma_s r4 - r2) + G_u^T a + K_ux q
template <bool kLDS, int kT>
__device__ __forceinline__ void step_rhs_body(const DP& d, int bx_, int by_, int gx_, const double* r1x, const double* r2,
                                                 const double* r3, const double* r4,
                                                 const double* ss) {
  extern __shared__ double smem[];
  const int k = bx_, tid = threadIdx.x;
  const StepView w = step_view<kLDS>(d, k, smem, r1x, r3, r2, r4, ss, nullptr);
  const int nx = d.nx, nu = d.nu;
  double* rh1 = w.v2;  // rhat1; the global copy is kept for the recovery
  double* q = w.v0;
  double* a = w.v1;
  double* grh1 = d.rhat1 + (long long)k * nx;
  for (int r = tid; r < d.m; r += kT) w.wv[r] = w.ss[r] * w.r4[r] - w.r2[r];
  __syncthreads();
  for (int i = tid; i < nx; i += kT) {
    const int pi = d.perm[i];
    double acc = w.ra[pi];
    const int j1 = d.ht_ptr[i + 1];
    for (int j = d.ht_ptr[i]; j < j1; ++j) acc = fma(w.hv[d.ht_pos[j]], w.wv[d.ht_row[j]], acc);
    rh1[i] = acc;
    q[i] = w.r3[pi];
  }
  __syncthreads();
  in_sweep_group<kLDS>([&](int gl, auto sync) { solve_fwd<kLDS>(d, w, q, gl, sync); });
  for (int i = tid; i < nx; i += kT) {
    double acc = rh1[i];
    const int e1 = d.k_usplit[i];
    for (int e = d.k_ptr[i]; e < e1; ++e) acc = fma(-w.Kv[e], q[d.k_col[e]], acc);
    a[i] = acc * w.invd[i];
    if (kLDS) grh1[i] = rh1[i];
  }
  __syncthreads();
  in_sweep_group<kLDS>([&](int gl, auto sync) { solve_adj_scaled<kLDS>(d, w, a, gl, sync); });
  for (int c = tid; c < nu; c += kT) {
    const int v = nx + c;
    double acc = 0.0;
    for (int j = d.ht_ptr[v]; j < d.ht_ptr[v + 1]; ++j) acc = fma(-w.hv[d.ht_pos[j]], w.wv[d.ht_row[j]], acc);
    for (int j = d.guc_ptr[c]; j < d.guc_ptr[c + 1]; ++j) acc = fma(w.guv[d.guc_pos[j]], a[d.guc_row[j]], acc);
    for (int e = d.k_ptr[v]; e < d.k_usplit[v]; ++e) acc = fma(w.Kv[e], q[d.k_col[e]], acc);
    d.rpart[(long long)k * nu + c] = acc;
  }
}

template <bool kLDS, int kT>
__global__ __launch_bounds__(kT) void k_step_rhs(DP d, const double* r1x, const double* r2,
                                                 const double* r3, const double* r4,
                                                 const double* ss) {
  step_rhs_body<kLDS, kT>(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, r1x, r2, r3, r4, ss);
}

// Recovery of one scenario (propositions "Reduction" and "Condensed KKT system"):
//   p_x = -G_x^-1 (r3 + G_u p_u), p_y = -G_x^-T (rhat1 + K_xx p_x + K_xu p_u),
//   p_s = -(r4 + H p_d), p_z = Sigma_s (H p_d + r4) - r2
template <bool kLDS, int kT>
__device__ __forceinline__ void step_recover_body(const DP& d, int bx_, int by_, int gx_, const double* r2, const double* r3,
                                                     const double* r4, const double* ss,
                                                     const double* pu, double* px, double* ps,
                                                     double* py, double* pz) {
  extern __shared__ double smem[];
  const int k = bx_, tid = threadIdx.x;
  const StepView w = step_view<kLDS>(d, k, smem, d.rhat1, r3, r2, r4, ss, pu);
  const int nx = d.nx;
  double* xv = w.v0;
  double* yv = w.v1;
  for (int i = tid; i < nx; i += kT) {
    double acc = w.r3[d.perm[i]];
    const int e1 = d.gu_ptr[i + 1];
    for (int e = d.gu_ptr[i]; e < e1; ++e) acc = fma(w.guv[e], w.pu[d.gu_col[e]], acc);
    xv[i] = -acc;
  }
  __syncthreads();
  in_sweep_group<kLDS>([&](int gl, auto sync) { solve_fwd<kLDS>(d, w, xv, gl, sync); });
  for (int i = tid; i < nx; i += kT) {
    px[(long long)k * nx + d.perm[i]] = xv[i];
    double acc = w.ra[i];
    const int e1 = d.k_ptr[i + 1];
    for (int e = d.k_ptr[i]; e < e1; ++e) {
      const int cc = d.k_col[e];
      acc = fma(w.Kv[e], cc < nx ? xv[cc] : w.pu[cc - nx], acc);
    }
    yv[i] = -acc * w.invd[i];
  }
  __syncthreads();
  in_sweep_group<kLDS>([&](int gl, auto sync) { solve_adj_scaled<kLDS>(d, w, yv, gl, sync); });
  for (int i = tid; i < nx; i += kT) py[(long long)k * nx + d.perm[i]] = yv[i];
  for (int r = tid; r < d.m; r += kT) {
    double hp = 0.0;
    const int e1 = d.h_ptr[r + 1];
    for (int e = d.h_ptr[r]; e < e1; ++e) {
      const int cc = d.h_col[e];
      hp = fma(w.hv[e], cc < nx ? xv[cc] : w.pu[cc - nx], hp);
    }
    ps[(long long)k * d.m + r] = -(w.r4[r] + hp);
    pz[(long long)k * d.m + r] = w.ss[r] * (hp + w.r4[r]) - w.r2[r];
  }
}

template <bool kLDS, int kT>
__global__ __launch_bounds__(kT) void k_step_recover(DP d, const double* r2, const double* r3,
                                                     const double* r4, const double* ss,
                                                     const double* pu, double* px, double* ps,
                                                     double* py, double* pz) {
  step_recover_body<kLDS, kT>(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, r2, r3, r4, ss, pu, px, ps, py, pz);
}

// ------------------------------------- step of the stacked variant
// The stacked reduction leaves Z = [T; I], T = -G_x^-1 G_u (internal row
// order, row pitch nu_pad), in HBM.  With it G_u^T G_x^-T b = -T^T b and
// G_x^-1 G_u p_u = -T p_u, so each step kernel keeps one sparse solve: the
// right-hand side keeps q = G_x^-1 r3, the recovery keeps p_y.  Wavefront 0
// runs that solve on LDS data while the other wavefronts compute the terms
// that do not depend on it; the dense products with T read Z with
// consecutive lanes on consecutive columns.

// the sweep-group view of the staged factor and schedule blob
__device__ __forceinline__ StepView sweep_view(const DP& d, double* lu, unsigned* ue) {
  StepView w{};
  w.lu = lu;
  w.invd = lu + d.nnz_f;
  unsigned* de = ue + 2 * d.n_sent;
  int* ip = reinterpret_cast<int*>(de + 2 * d.n_sent);
  w.uptr = ip;
  w.dptr = ip + d.nph_u * kGroupLds + 1;
  w.umax = w.dptr + d.nph_d * kGroupLds + 1;
  w.dmax = w.umax + d.nph_u;
  w.uent = ue;
  w.dent = de;
  return w;
}

// out[c] = sum_i Z[i][c] b[i] for c < nu; kT threads as row slices x columns,
// partial sums through red[kT + nu] (LDS), one barrier inside.  Each thread
// keeps kTtRows loads of its column in flight.
constexpr int kTtRows = 16;

// entries of a sparse row (K, or H^T) whose loads the step kernels issue
// together before adding their terms in row order
constexpr int kRowBatch = 8;

template <int kT>
__device__ __forceinline__ void dense_tt_times(const DP& d, const double* __restrict__ Zk,
                                               const double* b, double* red) {
  const int nu = d.nu, nx = d.nx, ld = d.nu_pad, tid = threadIdx.x;
  const bool wide = nu >= kT;
  const int ns = wide ? 1 : kT / nu;
  const int s = wide ? 0 : tid / nu;
  if (s < ns) {
    for (int c = wide ? tid : tid - s * nu; c < nu; c += wide ? kT : nu) {
      double a[kTtRows];
#pragma unroll
      for (int u = 0; u < kTtRows; ++u) a[u] = 0.0;
      for (int i0 = s; i0 < nx; i0 += kTtRows * ns) {
        double z[kTtRows];
#pragma unroll
        for (int u = 0; u < kTtRows; ++u) {
          const int i = i0 + u * ns;
          z[u] = i < nx ? Zk[(long long)i * ld + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kTtRows; ++u) {
          const int i = i0 + u * ns;
          if (i < nx) a[u] = fma(z[u], b[i], a[u]);
        }
      }
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < kTtRows; ++u) acc += a[u];
      red[s * nu + c] = acc;
    }
  }
  __syncthreads();
}

template <int kT>
__device__ __forceinline__ void step_rhs2_body(const DP& d, int bx_, int by_, int gx_, const double* r1x, const double* r2,
                                                  const double* r3, const double* r4,
                                                  const double* ss) {
  extern __shared__ double smem[];
  const int k = bx_, tid = threadIdx.x;
  const int nx = d.nx, nu = d.nu, m = d.m, nf = d.nnz_f;
  double* lu = smem;
  double* q = lu + nf + nx;
  double* b = q + nx;
  double* part = b + nx;
  double* red = part + nu;
  unsigned* ue = reinterpret_cast<unsigned*>(red + kT + nu);
  const ChainPos cp = chain_positions<false>(d, tid);
  stage_copy(lu, lu_of(d, k), nf + nx, tid, kT);
  stage_words(ue, d.blob_stp, d.blob_stp_words, tid, kT);
  const double* r3k = r3 + (long long)k * nx;
  for (int i = tid; i < nx; i += kT) q[i] = r3k[d.perm[i]];
  __syncthreads();
  if (tid < 64) {
    solve_fwd<true>(d, sweep_view(d, lu, ue), q, tid, [] { wave_sync(); }, cp);
  } else {
    // rhat1 = r1x + H_x^T w and H_u^T w, with w = Sigma_s r4 - r2 formed per use
    const double* hv = d.EV + (long long)k * d.n_ev + d.off_h;
    const double* ssk = ss + (long long)k * m;
    const double* r2k = r2 + (long long)k * m;
    const double* r4k = r4 + (long long)k * m;
    const double* r1k = r1x + (long long)k * nx;
    for (int v = tid - 64; v < nx + nu; v += kT - 64) {
      double acc = v < nx ? r1k[d.perm[v]] : 0.0;
      const int j1 = d.ht_ptr[v + 1];
      for (int j = d.ht_ptr[v]; j < j1; j += kRowBatch) {
        double hj[kRowBatch], wj[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          const int jj = min(j + u, j1 - 1), r = d.ht_row[jj];
          hj[u] = hv[d.ht_pos[jj]];
          wj[u] = ssk[r] * r4k[r] - r2k[r];
        }
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          if (j + u < j1) acc = fma(hj[u], wj[u], acc);
      }
      if (v < nx) b[v] = acc;
      else part[v - nx] = -acc;
    }
  }
  __syncthreads();
  // b = rhat1 - K_xx q; rhat1 and q are kept for the recovery
  const double* Kk = d.K + (long long)k * d.nnz_k;
  double* grh1 = d.rhat1 + (long long)k * nx;
  double* gq = d.qbuf + (long long)k * nx;
  for (int i = tid; i < nx; i += kT) {
    const double rh = b[i];
    grh1[i] = rh;
    gq[i] = q[i];
    double acc = rh;
    const int e1 = d.k_usplit[i];
    for (int e = d.k_ptr[i]; e < e1; e += kRowBatch) {
      double kv[kRowBatch];
      int kc[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int ee = min(e + u, e1 - 1);
        kv[u] = Kk[ee];
        kc[u] = d.k_col[ee];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (e + u < e1) acc = fma(-kv[u], q[kc[u]], acc);
    }
    b[i] = acc;
  }
  __syncthreads();
  dense_tt_times<kT>(d, d.Zst + (long long)k * d.nz * d.nu_pad, b, red);
  // rpart = -H_u^T w + K_ux q - T^T b
  const int ns = nu >= kT ? 1 : kT / nu;
  for (int c = tid; c < nu; c += kT) {
    const int v = nx + c;
    double acc = part[c];
    const int e1 = d.k_usplit[v];
    for (int e = d.k_ptr[v]; e < e1; e += kRowBatch) {
      double kv[kRowBatch];
      int kc[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int ee = min(e + u, e1 - 1);
        kv[u] = Kk[ee];
        kc[u] = d.k_col[ee];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (e + u < e1) acc = fma(kv[u], q[kc[u]], acc);
    }
    double tb = 0.0;
    for (int s = 0; s < ns; ++s) tb += red[s * nu + c];
    d.rpart[(long long)k * nu + c] = acc - tb;
  }
}

template <int kT>
__global__ __launch_bounds__(kT) void k_step_rhs2(DP d, const double* r1x, const double* r2,
                                                  const double* r3, const double* r4,
                                                  const double* ss) {
  step_rhs2_body<kT>(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, r1x, r2, r3, r4, ss);
}

constexpr int kPxRows = 4;     // rows of T per 16-lane group in flight
constexpr int kPxChunks = 8;   // 16-column chunks of a row per pass
constexpr int kKxPre = 16;     // entries of a K_x row loaded ahead

template <int kT>
__device__ __forceinline__ void step_recover2_body(const DP& d, int bx_, int by_, int gx_, const double* r2, const double* r3,
                                                      const double* r4, const double* ss,
                                                      const double* pu, double* px, double* ps,
                                                      double* py, double* pz) {
  extern __shared__ double smem[];
  const int k = bx_, tid = threadIdx.x;
  const int nx = d.nx, nu = d.nu, m = d.m, nf = d.nnz_f;
  double* lu = smem;
  double* xv = lu + nf + nx;
  double* yv = xv + nx;
  double* spu = yv + nx;
  unsigned* ue = reinterpret_cast<unsigned*>(spu + nu + kT + nu);
  const double* Kk = d.K + (long long)k * d.nnz_k;
  // loaded ahead: the chain positions of the adjoint solve and the extent of
  // this thread's first K_x row
  const ChainPos cp = chain_positions<true>(d, tid);
  const int ke0 = tid < nx ? d.k_ptr[tid] : 0, ke1 = tid < nx ? d.k_ptr[tid + 1] : 0;
  const double* grh1 = d.rhat1 + (long long)k * nx;
  const double rh = tid < nx ? grh1[tid] : 0.0;
  stage_copy(lu, lu_of(d, k), nf + nx, tid, kT);
  stage_words(ue, d.blob_stp, d.blob_stp_words, tid, kT);
  for (int c = tid; c < nu; c += kT) spu[c] = pu[c];
  __syncthreads();
  // the first K_x row's columns and values, in flight during p_x
  int kc[kKxPre];
  double kv[kKxPre];
#pragma unroll
  for (int u = 0; u < kKxPre; ++u) {
    const bool in = ke0 + u < ke1;
    kc[u] = in ? d.k_col[ke0 + u] : 0;
    kv[u] = in ? Kk[ke0 + u] : 0.0;
  }
  // p_x = -q + T p_u: 16-lane groups, kPxRows rows each (rows g + 16 r of the
  // batch), columns across the group, all of a batch's loads issued first
  {
    const double* Zk = d.Zst + (long long)k * d.nz * d.nu_pad;
    const double* gq = d.qbuf + (long long)k * nx;
    constexpr int kG = kT / 16;
    const int g = tid >> 4, l = tid & 15;
    for (int i0 = g; i0 < nx; i0 += kPxRows * kG) {
      double acc[kPxRows], qv[kPxRows];
#pragma unroll
      for (int r = 0; r < kPxRows; ++r) {
        acc[r] = 0.0;
        qv[r] = i0 + r * kG < nx ? gq[i0 + r * kG] : 0.0;
      }
      for (int c0 = 0; c0 < nu; c0 += 16 * kPxChunks) {
        double z[kPxRows][kPxChunks];
#pragma unroll
        for (int r = 0; r < kPxRows; ++r) {
          const int i = i0 + r * kG;
#pragma unroll
          for (int t = 0; t < kPxChunks; ++t) {
            const int c = c0 + l + 16 * t;
            z[r][t] = i < nx && c < nu ? Zk[(long long)i * d.nu_pad + c] : 0.0;
          }
        }
#pragma unroll
        for (int t = 0; t < kPxChunks; ++t) {
          const int c = c0 + l + 16 * t;
          const double p = c < nu ? spu[c] : 0.0;
#pragma unroll
          for (int r = 0; r < kPxRows; ++r) acc[r] = fma(z[r][t], p, acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < kPxRows; ++r) {
        double a = acc[r];
        a += __shfl_xor(a, 8, 16);
        a += __shfl_xor(a, 4, 16);
        a += __shfl_xor(a, 2, 16);
        a += __shfl_xor(a, 1, 16);
        const int i = i0 + r * kG;
        if (l == 0 && i < nx) {
          const double x = a - qv[r];
          xv[i] = x;
          px[(long long)k * nx + d.perm[i]] = x;
        }
      }
    }
  }
  __syncthreads();
  // p_y = -G_x^-T (rhat1 + K_x. [p_x; p_u]), prescaled by 1/u_ii
  const double* invd = lu + nf;
  for (int i = tid; i < nx; i += kT) {
    double acc;
    int e, e1;
    if (i == tid) {
      acc = rh;
#pragma unroll
      for (int u = 0; u < kKxPre; ++u)
        if (u < ke1 - ke0) acc = fma(kv[u], kc[u] < nx ? xv[kc[u]] : spu[kc[u] - nx], acc);
      e = ke0 + kKxPre;
      e1 = ke1;
    } else {
      acc = grh1[i];
      e = d.k_ptr[i];
      e1 = d.k_ptr[i + 1];
    }
    for (; e < e1; e += kRowBatch) {
      double kv2[kRowBatch];
      int kc2[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int ee = min(e + u, e1 - 1);
        kv2[u] = Kk[ee];
        kc2[u] = d.k_col[ee];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (e + u < e1) acc = fma(kv2[u], kc2[u] < nx ? xv[kc2[u]] : spu[kc2[u] - nx], acc);
    }
    yv[i] = -acc * invd[i];
  }
  __syncthreads();
  if (tid < 64) {
    solve_adj_scaled<true>(d, sweep_view(d, lu, ue), yv, tid, [] { wave_sync(); }, cp);
  } else {
    // p_s = -(r4 + H p_d), p_z = Sigma_s (H p_d + r4) - r2, beside the solve
    const double* hv = d.EV + (long long)k * d.n_ev + d.off_h;
    const double* ssk = ss + (long long)k * m;
    const double* r2k = r2 + (long long)k * m;
    const double* r4k = r4 + (long long)k * m;
    for (int r = tid - 64; r < m; r += kT - 64) {
      double hp = 0.0;
      const int e1 = d.h_ptr[r + 1];
      for (int e = d.h_ptr[r]; e < e1; ++e) {
        const int cc = d.h_col[e];
        hp = fma(hv[e], cc < nx ? xv[cc] : spu[cc - nx], hp);
      }
      ps[(long long)k * m + r] = -(r4k[r] + hp);
      pz[(long long)k * m + r] = ssk[r] * (hp + r4k[r]) - r2k[r];
    }
  }
  __syncthreads();
  for (int i = tid; i < nx; i += kT) py[(long long)k * nx + d.perm[i]] = yv[i];
}

template <int kT>
__global__ __launch_bounds__(kT) void k_step_recover2(DP d, const double* r2, const double* r3,
                                                      const double* r4, const double* ss,
                                                      const double* pu, double* px, double* ps,
                                                      double* py, double* pz) {
  step_recover2_body<kT>(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, r2, r3, r4, ss, pu, px, ps, py, pz);
}

// rows nx .. nz of every scenario block of the stacked Z are the identity
__global__ void k_identity_rows(DP d) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * d.nu) return;
  const int k = (int)(t / d.nu), j = (int)(t % d.nu);
  d.Zst[((long long)k * d.nz + d.nx + j) * d.nu_pad + j] = 1.0;
}

hipError_t allow_lds(const void* fn, int* cur, long long need) {
  if (need <= *cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
  if (e == hipSuccess) *cur = (int)need;
  return e;
}

int ntiles(const DP& d) { return (d.nu + d.col_tile - 1) / d.col_tile; }

// ---- entry points: several instances (block b is block (blk[b].bx,
// blk[b].by) of instance blk[b].inst's own grid, blk[b].gx wide)
#define RKKT_MULTI_ARGS \
  const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its, const MultiBlk* __restrict__ blk
#define RKKT_MULTI_PROLOGUE                          \
  const MultiBlk mb = blk[blockIdx.x];               \
  const DP& d = dps[mb.inst];                        \
  const rkkt_iteration& it = its[mb.inst];           \
  (void)it;

template <bool kLDS, int kT, bool kUpdLds>
__global__ __launch_bounds__(kT) void k_refactor_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  refactor_body<kLDS, kT, kUpdLds>(d, mb.bx, mb.by, mb.gx);
}
template <bool kLDS, int kVar>
__global__ __launch_bounds__(kRT) void k_reduce_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  reduce_body<kLDS, kVar>(d, mb.bx, mb.by, mb.gx);
}
template <bool kLDS, int kVar>
__global__ __launch_bounds__(kRT) void k_reduce64_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  reduce64_body<kLDS, kVar>(d, mb.bx, mb.by, mb.gx);
}
template <bool kLDS, int kT>
__global__ __launch_bounds__(kT) void k_step_rhs_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  step_rhs_body<kLDS, kT>(d, mb.bx, mb.by, mb.gx, it.r1x, it.r2, it.r3, it.r4, it.sigma_s);
}
template <int kT>
__global__ __launch_bounds__(kT) void k_step_rhs2_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  step_rhs2_body<kT>(d, mb.bx, mb.by, mb.gx, it.r1x, it.r2, it.r3, it.r4, it.sigma_s);
}
template <bool kLDS, int kT>
__global__ __launch_bounds__(kT) void k_step_recover_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  step_recover_body<kLDS, kT>(d, mb.bx, mb.by, mb.gx, it.r2, it.r3, it.r4, it.sigma_s, it.pu, it.px, it.ps,
                              it.py, it.pz);
}
template <int kT>
__global__ __launch_bounds__(kT) void k_step_recover2_m(RKKT_MULTI_ARGS) {
  RKKT_MULTI_PROLOGUE
  step_recover2_body<kT>(d, mb.bx, mb.by, mb.gx, it.r2, it.r3, it.r4, it.sigma_s, it.pu, it.px, it.ps, it.py,
                         it.pz);
}

}  // namespace

hipError_t configure_lu_kernels(const DP& d) {
  static int c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0, c8 = 0;
  const LdsSizes z = sizes_of(d);
  hipError_t e = hipSuccess;
  if (d.lds_grp) {
    if (d.upd_lds) e = allow_lds((const void*)k_refactor<true, kGT, true>, &c1, refactor_lds_bytes(z));
    else e = allow_lds((const void*)k_refactor<true, kGT, false>, &c6, refactor_lds_bytes(z));
  }
  if (e == hipSuccess && d.lds_stp) {
    e = allow_lds((const void*)k_step_rhs<true, kGT>, &c3, step_lds_bytes(z));
    if (e == hipSuccess) e = allow_lds((const void*)k_step_recover<true, kGT>, &c4, step_lds_bytes(z));
    if (e == hipSuccess && d.variant == 2) {
      static int c9 = 0, c10 = 0;
      e = allow_lds((const void*)k_step_rhs2<kGT>, &c9, step2_lds_bytes(z, kGT));
      if (e == hipSuccess) e = allow_lds((const void*)k_step_recover2<kGT>, &c10, step2_lds_bytes(z, kGT));
    }
  }
  if (e == hipSuccess && d.lds_red) {
    if (d.col_tile == kW64) {
      if (d.variant == 2) e = allow_lds((const void*)k_reduce64<true, 2>, &c7, reduce_lds_bytes(z));
      else e = allow_lds((const void*)k_reduce64<true, 1>, &c8, reduce_lds_bytes(z));
    } else {
      if (d.variant == 2) e = allow_lds((const void*)k_reduce<true, 2>, &c5, reduce_lds_bytes(z));
      else e = allow_lds((const void*)k_reduce<true, 1>, &c2, reduce_lds_bytes(z));
    }
  }
  return e;
}

void launch_identity_rows(const DP& d, hipStream_t s) {
  const long long n = (long long)d.N * d.nu;
  k_identity_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d);
}

void launch_refactor(const DP& d, hipStream_t s) {
  const unsigned grid = (d.N + d.spw - 1) / d.spw;
  const size_t lds = refactor_lds_bytes(sizes_of(d));
  if (d.lds_grp && d.upd_lds)
    k_refactor<true, kGT, true><<<grid, kGroupLds * d.spw, lds, s>>>(d);
  else if (d.lds_grp)
    k_refactor<true, kGT, false><<<grid, kGroupLds * d.spw, lds, s>>>(d);
  else
    k_refactor<false, kRT, false><<<d.N, kRT, 0, s>>>(d);
}

void launch_reduce(const DP& d, hipStream_t s) {
  dim3 grid(ntiles(d), d.N);
  // LDS mode: the staged data; global mode: only the chain block's values
  const size_t lds = d.lds_red ? reduce_lds_bytes(sizes_of(d)) : 8 * (size_t)d.chain_t * d.chain_t;
  if (d.col_tile == kW64) {
    if (d.variant == 2) {
      if (d.lds_red) k_reduce64<true, 2><<<grid, kRT, lds, s>>>(d);
      else k_reduce64<false, 2><<<grid, kRT, lds, s>>>(d);
    } else {
      if (d.lds_red) k_reduce64<true, 1><<<grid, kRT, lds, s>>>(d);
      else k_reduce64<false, 1><<<grid, kRT, lds, s>>>(d);
    }
    return;
  }
  if (d.variant == 2) {
    if (d.lds_red) k_reduce<true, 2><<<grid, kRT, lds, s>>>(d);
    else k_reduce<false, 2><<<grid, kRT, lds, s>>>(d);
  } else {
    if (d.lds_red) k_reduce<true, 1><<<grid, kRT, lds, s>>>(d);
    else k_reduce<false, 1><<<grid, kRT, lds, s>>>(d);
  }
}

// the stacked variant's one-solve step kernels (LDS mode)
static bool step2(const DP& d) { return d.variant == 2 && d.lds_stp; }

void launch_step_rhs(const DP& d, const double* r1x, const double* r2, const double* r3,
                     const double* r4, const double* ss, hipStream_t s) {
  if (step2(d))
    k_step_rhs2<kGT><<<d.N, kGT, step2_lds_bytes(sizes_of(d), kGT), s>>>(d, r1x, r2, r3, r4, ss);
  else if (d.lds_stp)
    k_step_rhs<true, kGT><<<d.N, kGT, step_lds_bytes(sizes_of(d)), s>>>(d, r1x, r2, r3, r4, ss);
  else
    k_step_rhs<false, kRT><<<d.N, kRT, 0, s>>>(d, r1x, r2, r3, r4, ss);
}

void launch_step_recover(const DP& d, const double* r2, const double* r3, const double* r4,
                         const double* ss, const double* pu, double* px, double* ps, double* py,
                         double* pz, hipStream_t s) {
  if (step2(d))
    k_step_recover2<kGT><<<d.N, kGT, step2_lds_bytes(sizes_of(d), kGT), s>>>(d, r2, r3, r4, ss, pu,
                                                                            px, ps, py, pz);
  else if (d.lds_stp)
    k_step_recover<true, kGT><<<d.N, kGT, step_lds_bytes(sizes_of(d)), s>>>(d, r2, r3, r4, ss, pu, px,
                                                                           ps, py, pz);
  else
    k_step_recover<false, kRT><<<d.N, kRT, 0, s>>>(d, r2, r3, r4, ss, pu, px, ps, py, pz);
}

}  // namespace rkkt

namespace rkkt {

// the launches of launch_refactor, launch_reduce, launch_step_rhs and
// launch_step_recover.  Variants: refactor 0 LDS with staged updates, 1 LDS,
// 2 global; reduce (64-column or narrow tiles) 2 (lds ? 1 : 0) + (variant
// == 2); steps 0 one-solve (stacked variant), 1 LDS, 2 global.
void launches_lu(const DP& d, std::vector<Launch>& out) {
  {
    const LdsSizes z = sizes_of(d);
    if (d.lds_grp)
      out.push_back(Launch{kStRefactor * 4096, kKRefactor, d.upd_lds ? 0 : 1, (d.N + d.spw - 1) / d.spw, 1,
                           kGroupLds * d.spw, 0, refactor_lds_bytes(z)});
    else
      out.push_back(Launch{kStRefactor * 4096, kKRefactor, 2, d.N, 1, kRT, 0, 0});
    const long long lds = d.lds_red ? reduce_lds_bytes(z) : 8LL * d.chain_t * d.chain_t;
    out.push_back(Launch{kStReduce * 4096, d.col_tile == kW64 ? kKReduce64 : kKReduce,
                         2 * (d.lds_red ? 1 : 0) + (d.variant == 2 ? 1 : 0), ntiles(d), d.N, kRT, 0, lds});
    if (step2(d)) {
      out.push_back(Launch{kStStepRhs * 4096, kKStepRhs2, 0, d.N, 1, kGT, 0, step2_lds_bytes(z, kGT)});
      out.push_back(Launch{kStRecover * 4096, kKStepRec2, 0, d.N, 1, kGT, 0, step2_lds_bytes(z, kGT)});
    } else if (d.lds_stp) {
      out.push_back(Launch{kStStepRhs * 4096, kKStepRhs, 1, d.N, 1, kGT, 0, step_lds_bytes(z)});
      out.push_back(Launch{kStRecover * 4096, kKStepRec, 1, d.N, 1, kGT, 0, step_lds_bytes(z)});
    } else {
      out.push_back(Launch{kStStepRhs * 4096, kKStepRhs, 2, d.N, 1, kRT, 0, 0});
      out.push_back(Launch{kStRecover * 4096, kKStepRec, 2, d.N, 1, kRT, 0, 0});
    }
  }
}

hipError_t multi_lu(const Launch& l, unsigned nblk, long long lds, const DP* dps, const rkkt_iteration* its,
                    const MultiBlk* blk, hipStream_t s, bool prepare, bool* handled) {
  *handled = true;
  const size_t L = (size_t)lds;
  const unsigned T = (unsigned)l.threads;
  // one dynamic-LDS limit per multi-instance kernel, raised as needed
  static int cur[32] = {};
  auto go = [&](const void* fn, int slot, auto launch) -> hipError_t {
    if (prepare) return allow_lds(fn, &cur[slot], lds);
    launch();
    return hipSuccess;
  };
  switch (l.kernel) {
    case kKRefactor:
      if (l.variant == 0)
        return go((const void*)k_refactor_m<true, kGT, true>, 0,
                  [&] { k_refactor_m<true, kGT, true><<<nblk, T, L, s>>>(dps, its, blk); });
      if (l.variant == 1)
        return go((const void*)k_refactor_m<true, kGT, false>, 1,
                  [&] { k_refactor_m<true, kGT, false><<<nblk, T, L, s>>>(dps, its, blk); });
      return go((const void*)k_refactor_m<false, kRT, false>, 2,
                [&] { k_refactor_m<false, kRT, false><<<nblk, T, L, s>>>(dps, its, blk); });
    case kKReduce64:
      switch (l.variant) {
        case 0: return go((const void*)k_reduce64_m<false, 1>, 3, [&] { k_reduce64_m<false, 1><<<nblk, T, L, s>>>(dps, its, blk); });
        case 1: return go((const void*)k_reduce64_m<false, 2>, 4, [&] { k_reduce64_m<false, 2><<<nblk, T, L, s>>>(dps, its, blk); });
        case 2: return go((const void*)k_reduce64_m<true, 1>, 5, [&] { k_reduce64_m<true, 1><<<nblk, T, L, s>>>(dps, its, blk); });
        default: return go((const void*)k_reduce64_m<true, 2>, 6, [&] { k_reduce64_m<true, 2><<<nblk, T, L, s>>>(dps, its, blk); });
      }
    case kKReduce:
      switch (l.variant) {
        case 0: return go((const void*)k_reduce_m<false, 1>, 7, [&] { k_reduce_m<false, 1><<<nblk, T, L, s>>>(dps, its, blk); });
        case 1: return go((const void*)k_reduce_m<false, 2>, 8, [&] { k_reduce_m<false, 2><<<nblk, T, L, s>>>(dps, its, blk); });
        case 2: return go((const void*)k_reduce_m<true, 1>, 9, [&] { k_reduce_m<true, 1><<<nblk, T, L, s>>>(dps, its, blk); });
        default: return go((const void*)k_reduce_m<true, 2>, 10, [&] { k_reduce_m<true, 2><<<nblk, T, L, s>>>(dps, its, blk); });
      }
    case kKStepRhs2:
      return go((const void*)k_step_rhs2_m<kGT>, 11, [&] { k_step_rhs2_m<kGT><<<nblk, T, L, s>>>(dps, its, blk); });
    case kKStepRec2:
      return go((const void*)k_step_recover2_m<kGT>, 12,
                [&] { k_step_recover2_m<kGT><<<nblk, T, L, s>>>(dps, its, blk); });
    case kKStepRhs:
      if (l.variant == 1)
        return go((const void*)k_step_rhs_m<true, kGT>, 13, [&] { k_step_rhs_m<true, kGT><<<nblk, T, L, s>>>(dps, its, blk); });
      return go((const void*)k_step_rhs_m<false, kRT>, 14, [&] { k_step_rhs_m<false, kRT><<<nblk, T, L, s>>>(dps, its, blk); });
    case kKStepRec:
      if (l.variant == 1)
        return go((const void*)k_step_recover_m<true, kGT>, 15,
                  [&] { k_step_recover_m<true, kGT><<<nblk, T, L, s>>>(dps, its, blk); });
      return go((const void*)k_step_recover_m<false, kRT>, 16,
                [&] { k_step_recover_m<false, kRT><<<nblk, T, L, s>>>(dps, its, blk); });
    default:
      *handled = false;
      return hipSuccess;
  }
}

}  // namespace rkkt
