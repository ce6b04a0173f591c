// Device kernels of the tensor-product multigrid / CG solver for gfx950.
//
// Every kernel is HBM-bandwidth bound (well under 1 flop per byte), so the
// design is about data movement, not arithmetic: one lane owns one vertical
// column and marches up (and down) the column; columns of one colour are
// stored contiguously per level ("colour-split" layout, [colour][k][m]), so a
// wavefront's 64 lanes touch 64 consecutive doubles at every level k and the
// red/black sweeps read and write full cache lines.  The vertical
// coefficients depend on k (and the level) only, so every coefficient is a
// wave-uniform scalar load; nothing is stored per column (Sec. 6.2.1: the
// matrix is never stored).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ell {

constexpr int kBlock = 256;  // 4 wavefronts of 64 lanes

// Table slots of one level, each nz+1 long (see host-side construction).
// TPF/TQB: products of the forward / backward recurrence multipliers over
// each k-segment (see k_smooth_seg).
enum : int { TV = 0, TX = 1, TY = 2, TZ = 3, TIP = 4, TCF = 5, TPF = 6, TQB = 7, TSLOTS = 8 };

// Segments a column is split into along k: one wavefront per segment, so a
// block of kSeg wavefronts covers 64 columns.  The line smoother chooses its
// own segment count per level (more segments on small, latency-bound levels).
constexpr int kSeg = 4;
constexpr int kSegCols = 64;

__host__ __device__ inline int seg_len(int nz, int nseg = kSeg) { return (nz + nseg - 1) / nseg; }


// Geometry of one level in the colour-split layout.
struct Geo {
  int nx, ny, nz;
  int H;          // allocated columns per colour array = ceil(nx*ny/2)
  int ncol0;      // red columns
  int ncol1;      // black columns
  int hx2;        // nx/2 (nx > 1)
  int has_x;      // nx > 1: x faces exist
  int has_y;      // ny > 1
  int P;          // table stride = nz + 1
  int S;          // plane stride of a colour array (>= H, padded so that
                  // successive k-planes do not start on the same HBM channel)
  int nseg;       // k-segments per column used by the line smoother
  long long cs;   // colour stride (>= nz * S)
};

struct PcgState {
  // alpha: the last step length; alpha_prev: the one before (the solution
  // updates of two iterations are applied together)
  double kappa_old, alpha, alpha_prev, beta, r0_norm, b_norm, r_norm, thresh, true_r_norm;
  int iter, done, status, maxiter, flexible;
  int pending;  // a step length alpha waits for its residual update (set by F_ALPHA)
  // grid_barrier of the cooperative coarsest-level sweeps: arrivals,
  // generation, a timeout flag (zeroed when the grid is created)
  unsigned bar[4];
};

// The deferred solution updates of CG: iteration K's update u += alpha_K p_K
// waits for the operator step of a later iteration, which reads and writes u
// for two updates at once.  The steps of odd K >= 3 apply those of K - 2 and
// K - 1; the end of a solve after K iterations applies the rest (K even:
// K - 1 and K; K odd: K).  p_K lives in buffer dir_slot(K) of three: the
// step of K overwrites p_{K-3}, which was applied at step K - 1 or K - 2.
__host__ __device__ inline int deferred_updates(int K) { return K >= 3 && (K & 1) ? 2 : 0; }
__host__ __device__ inline int pending_at_end(int K) { return K <= 0 ? 0 : ((K & 1) ? 1 : 2); }
__host__ __device__ inline int dir_slot(int K) { return ((K % 3) + 3) % 3; }

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b mod 8);
// every grid here is a multiple of 8 blocks and this map gives each XCD a
// contiguous range of logical blocks, so neighbouring rows of columns (which
// share halo data) meet in the same L2.
__device__ __forceinline__ int logical_block() {
#ifdef ELL_NO_XCD_REMAP
  return blockIdx.x;
#else
  const int g8 = gridDim.x >> 3;
  return (blockIdx.x & 7) * g8 + (blockIdx.x >> 3);
#endif
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ void col_ij(const Geo &L, int c, int m, int &i, int &j) {
  if (L.nx > 1) {
    j = m / L.hx2;
    i = 2 * (m - j * L.hx2) + ((j + c) & 1);
  } else {
    i = 0;
    j = 2 * m + c;
  }
}

__device__ __forceinline__ int col_m(const Geo &L, int i, int j) {
  return L.nx > 1 ? j * L.hx2 + (i >> 1) : (j >> 1);
}

__device__ __forceinline__ bool is_done(const int *done) { return done != nullptr && *done != 0; }

// Index of the wavefront within the block, known to the compiler to be the
// same for all lanes (so values derived from it live in scalar registers and
// coefficient reads indexed by it stay scalar loads).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Sum over the 256 threads of a block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// A pointer that is the same for the whole block, re-derived through
// readfirstlane and the global address space: the value sits in scalar
// registers and memory instructions through it are global (not flat) ones.
// The batch kernels use it for pointers read from grid descriptors.  The
// result carries no aliasing facts of the original, so the compiler keeps its
// loads on the program-order side of a memory clobber: the tiled smoother
// relies on that to issue a whole chunk's loads before its first level runs.
template <typename T>
__device__ __forceinline__ T *gp(T *p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  auto *g = (__attribute__((address_space(1))) T *)(((unsigned long long)hi << 32) | lo);
  return (T *)g;
}

// The same for data that no kernel writes while it runs (the coefficient
// tables): through the constant address space, the loads of a uniform index
// stay scalar loads even where stores through other re-derived pointers, or a
// memory clobber, stand between the kernel's start and the load.
template <typename T>
__device__ __forceinline__ const T *cp(const T *p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  auto *c = (const __attribute__((address_space(4))) T *)(((unsigned long long)hi << 32) | lo);
  return (const T *)c;
}

// Streaming (nontemporal) accesses for data a kernel touches exactly once:
// finest-level vectors are far larger than the L2 and the Infinity Cache, so
// keeping them out of the caches leaves room for the data that is reused (the
// neighbour columns of the stencils).
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
  const nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(double2 *p, double2 v) {
  const nt_d2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, (nt_d2 *)p);
}
// NT is a template argument: with a run-time flag the compiler merges the two
// loads into one and drops the streaming hint.
template <bool NT, typename T>
__device__ __forceinline__ T ld_s(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Neighbour columns (colour 1 - c) of column (i, j) in the split layout.
struct Nbr {
  int w, e, s, n;
};

__device__ __forceinline__ Nbr neighbours(const Geo &L, int i, int j) {
  Nbr r{0, 0, 0, 0};
  if (L.has_x) {
    r.w = col_m(L, wrapi(i - 1, L.nx), j);
    r.e = col_m(L, wrapi(i + 1, L.nx), j);
  }
  if (L.has_y) {
    r.s = col_m(L, i, wrapi(j - 1, L.ny));
    r.n = col_m(L, i, wrapi(j + 1, L.ny));
  }
  return r;
}

// Number of levels whose loads are issued together before they are used:
// the column recurrences are sequential in k, so the memory-level
// parallelism of a lane comes from fetching a chunk of levels at once.
constexpr int kChunk = 8;

// -------------------------------------------------------------------------
// One colour of block red/black SOR (Sec. 4.2 eq. BlockRBSOR): per column of
// colour c, g_k = b_k + Tx_k (u_W + u_E) + Ty_k (u_S + u_N) with the other
// colour's values, then the tridiagonal column solve (Thomas, Appendix B)
// with per-level shared factors: y_k = (g_k + T_{k-1/2} y_{k-1}) / p_k
// forward, w_k = y_k + (T_{k+1/2}/p_k) w_{k+1} backward.  The forward values y
// are parked in the output column itself (rho = 1) and read back on the way
// down, so no per-lane array is needed and occupancy stays high.
//   bo: b of colour c; uo: u of colour 1-c; own: u of colour c (distinct
//   arrays, so loads can run ahead of the stores).
// FINE marks launches on the finest level (a separate kernel symbol, so that
// profiles attribute the dominant launches to it alone).  HXY: both
// horizontal directions have faces (every level but degenerate 1-wide ones).
// -------------------------------------------------------------------------
// C3 (horizontally varying vertical coefficients): every column has its own
// faces and Thomas factors, read from the level's split-layout fields tz3
// (T_{k-1/2}, zero at k = 0), ip3 (1/p_k) and cf3 (T_{k+1/2}/p_k) instead of
// the table's shared columns.
template <typename R, bool ZERO, bool RHO1, bool FINE, bool HXY, bool C3 = false>
__global__ __launch_bounds__(kBlock) void k_smooth(Geo L, const R *__restrict__ tab, int c,
                                                   const R *__restrict__ bo,
                                                   const R *__restrict__ uo,
                                                   R *__restrict__ own, R *__restrict__ ybuf,
                                                   R rho, const int *__restrict__ done,
                                                   const R *__restrict__ tz3 = nullptr,
                                                   const R *__restrict__ ip3 = nullptr,
                                                   const R *__restrict__ cf3 = nullptr) {
  if (is_done(done)) return;
  const int m = logical_block() * kBlock + threadIdx.x;
  const int ncol = c ? L.ncol1 : L.ncol0;
  if (m >= ncol) return;
  int i, j;
  col_ij(L, c, m, i, j);
  const Nbr nb = ZERO ? Nbr{0, 0, 0, 0} : neighbours(L, i, j);
  const bool hx = HXY || L.has_x, hy = HXY || L.has_y;
  const long long H = L.S;
  bo += m;
  own += m;
  const R *__restrict__ uw = uo + nb.w;
  const R *__restrict__ ue = uo + nb.e;
  const R *__restrict__ us = uo + nb.s;
  const R *__restrict__ un = uo + nb.n;
  R *ys = RHO1 ? own : ybuf + m;
  const R *__restrict__ tx = tab + TX * L.P;
  const R *__restrict__ ty = tab + TY * L.P;
  const R *__restrict__ tz = tab + TZ * L.P;
  const R *__restrict__ ip = tab + TIP * L.P;
  const R *__restrict__ cf = tab + TCF * L.P;
  const int nz = L.nz;
  // per-column fields of this column (C3)
  const long long oc3 = (long long)c * L.cs + m;
  auto tzb = [&](int k) -> R { if constexpr (C3) return tz3[oc3 + (long long)k * H]; else return tz[k]; };
  auto ipk = [&](int k) -> R { if constexpr (C3) return ip3[oc3 + (long long)k * H]; else return ip[k]; };
  auto cfk = [&](int k) -> R { if constexpr (C3) return cf3[oc3 + (long long)k * H]; else return cf[k]; };

  auto gval = [&](int k) -> R {
    const long long o = (long long)k * H;
    R v = bo[o];
    if (!ZERO) {
      if (hx) v = v + tx[k] * (uw[o] + ue[o]);
      if (hy) v = v + ty[k] * (us[o] + un[o]);
    }
    return v;
  };

  R yprev = R(0);
  int k = 0;
  for (; k + kChunk <= nz; k += kChunk) {
    R g[kChunk], a[kChunk], d[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      g[t] = gval(k + t);
      a[t] = tzb(k + t);
      d[t] = ipk(k + t);
    }
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      const R y = (g[t] + a[t] * yprev) * d[t];
      ys[(long long)(k + t) * H] = y;
      yprev = y;
    }
  }
  for (; k < nz; ++k) {
    const R y = (gval(k) + tzb(k) * yprev) * ipk(k);
    ys[(long long)k * H] = y;
    yprev = y;
  }

  R w = yprev;
  if (!RHO1) {
    const long long o = (long long)(nz - 1) * H;
    const R old = ZERO ? R(0) : own[o];
    own[o] = (R(1) - rho) * old + rho * w;
  }
  k = nz - 2;
  for (; k + 1 >= kChunk; k -= kChunk) {
    R y[kChunk], old[kChunk], e[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      y[t] = ys[(long long)(k - t) * H];
      old[t] = (RHO1 || ZERO) ? R(0) : own[(long long)(k - t) * H];
      e[t] = cfk(k - t);
    }
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      w = y[t] + e[t] * w;
      own[(long long)(k - t) * H] = RHO1 ? w : (R(1) - rho) * old[t] + rho * w;
    }
  }
  for (; k >= 0; --k) {
    const long long o = (long long)k * H;
    const R old = (RHO1 || ZERO) ? R(0) : own[o];
    w = ys[o] + cfk(k) * w;
    own[o] = RHO1 ? w : (R(1) - rho) * old + rho * w;
  }
}

// v of lane q (q wave-uniform) in every lane.
template <typename R>
__device__ __forceinline__ R lane_value(R v, int q) {
  if constexpr (sizeof(R) == 8) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, q);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), q);
    return __builtin_bit_cast(R, ((unsigned long long)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(R, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), q));
  }
}

// -------------------------------------------------------------------------
// The same half-sweep with each column split into kSeg segments along k, one
// wavefront per segment (k is uniform across a wavefront, so coefficients are
// scalar loads and every access is 64 consecutive elements).  The Thomas
// factors are shared by all columns, so the two triangular recurrences
//   forward  y_k = a_k y_{k-1} + g_k/p_k,   a_k = T_{k-1/2}/p_k
//   backward w_k = y_k + c_k w_{k+1},       c_k = T_{k+1/2}/p_k
// are evaluated per segment from a zero start and joined afterwards:
//   y_k = y_k(local) + Pf_k y_in,   Pf_k = prod_{i=start..k} a_i
//   w_k = w_k(local) + Qb_k w_in,   Qb_k = prod_{i=k..end-1} c_i
// with y_in / w_in the true values just below / above the segment, passed
// from segment to segment through LDS.  Pf and Qb are per-level tables.  The
// forward values stay in registers (SEG >= segment length).
// -------------------------------------------------------------------------
// TB: element type of b (the FP32 preconditioner reads the FP64 CG residual
// directly on the finest level).
// The rest of a segmented half-sweep once every segment has run its local
// forward recurrence (y[] local, prev = its last value): join the forward
// values across segments, run the local backward recurrence, join it, and
// write the column (rho = 1: the new values; else the relaxation).  xch: the
// block's exchange array [NSEG][kSegCols]; ow: the output column at level 0.
// DOT (rho = 1 only) also accumulates the CG inner products of the written
// values w: dsum[0] += b w with b from bl[t * 64 + lane] (level k0 + t), and
// with DOT = 2 dsum[1] += q w with q read from the column qo.
template <typename R, bool ZERO, bool RHO1, bool FINE, int SEG, int NSEG, int DOT = 0>
__device__ __forceinline__ void seg_join_store(R (&y)[SEG], R prev, R (*xch)[kSegCols], int sg, int lane,
                                               int k0, int k1, int len, int nz, int Ls,
                                               const R *__restrict__ pf, const R *__restrict__ cf,
                                               const R *__restrict__ qb, bool valid, R *__restrict__ ow,
                                               long long H, R rho, const double *bl = nullptr,
                                               const double *__restrict__ qo = nullptr,
                                               double *dsum = nullptr) {
  // Lane q < NSEG loads segment q's Pf at its last level and Qb at its first
  // (1 for an empty segment) before the barrier, and the joins take them
  // from that lane: their LDS reads issue together and only the multiply-adds
  // are sequential (segment q < sg joins forward, q > sg backward).
  R pfq = R(1), qbq = R(1);
  if (lane < NSEG) {
    const int s0 = min(lane * Ls, nz), e = min(s0 + Ls, nz);
    if (e > s0) {
      pfq = pf[e - 1];
      qbq = qb[s0];
    }
  }
  // join the forward recurrence across segments
  xch[sg][lane] = prev;
  __syncthreads();
  R yin = R(0);
#pragma unroll
  for (int q = 0; q < NSEG - 1; ++q) {
    const R cand = xch[q][lane] + lane_value(pfq, q) * yin;
    yin = q < sg ? cand : yin;
  }
  __syncthreads();
  // true y, then the local backward recurrence (in place)
  R nxt = R(0);
#pragma unroll
  for (int t = SEG - 1; t >= 0; --t) {
    if (t < len) {
      const int k = k0 + t;
      const R yt = y[t] + pf[k] * yin;
      nxt = yt + cf[k] * nxt;
      y[t] = nxt;
    }
  }
  xch[sg][lane] = nxt;  // local w at the segment's first level
  __syncthreads();
  R win = R(0);
#pragma unroll
  for (int q = NSEG - 1; q > 0; --q) {
    const R cand = xch[q][lane] + lane_value(qbq, q) * win;
    win = q > sg ? cand : win;
  }
  if (valid) {
#pragma unroll
    for (int c0 = 0; c0 < SEG; c0 += 8) {
      if (c0 < len) {
        R old[8];
        double qv[8];
        if (!RHO1 && !ZERO) {
#pragma unroll
          for (int t = 0; t < 8; ++t) old[t] = ow[(long long)min(k0 + c0 + t, k1 - 1) * H];
        }
        if constexpr (DOT == 2) {
#pragma unroll
          for (int t = 0; t < 8; ++t) qv[t] = __builtin_nontemporal_load(&qo[(long long)min(k0 + c0 + t, k1 - 1) * H]);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (c0 + t < len) {
            const int k = k0 + c0 + t;
            const R w = y[c0 + t] + qb[k] * win;
            const R o = (RHO1 || ZERO) ? R(0) : old[t];
            // plain stores also on the finest level: streaming stores measured
            // slower here
            ow[(long long)k * H] = RHO1 ? w : (R(1) - rho) * o + rho * w;
            if constexpr (DOT >= 1) dsum[0] += bl[(c0 + t) * 64 + lane] * (double)w;
            if constexpr (DOT == 2) dsum[1] += qv[t] * (double)w;
          }
        }
      }
    }
  }
}

// UPD (the first pre-smoothing pair of a CG preconditioner application, b
// being the CG residual of this colour, TB = double): b is first advanced to
// b - alpha q (alpha: the CG step length in st; qo: this colour's part of q)
// and written back to rw, and the block's partial sum of its squares goes to
// partial[pbase + lb] (the residual update and its norm, fused into the sweep).
template <typename R, bool ZERO, bool RHO1, bool FINE, int SEG, int NSEG, typename TB = R, bool UPD = false>
__device__ __forceinline__ void smooth_seg_body(Geo L, const R *__restrict__ tab, int c,
                                                          const TB *__restrict__ bo,
                                                          const R *__restrict__ uo,
                                                          R *__restrict__ own, R rho,
                                                          const int *__restrict__ done, int lb, int nblocks,
                                                          double *__restrict__ rw = nullptr,
                                                          const double *__restrict__ qo = nullptr,
                                                          const PcgState *__restrict__ st = nullptr,
                                                          double *__restrict__ partial = nullptr, int pbase = 0) {
  __shared__ R xch[NSEG][kSegCols];
  __shared__ double red[UPD ? NSEG : 1];
  if (is_done(done)) return;
  const int lane = threadIdx.x & 63;
  const int sg = wave_id();
  const int ncol = c ? L.ncol1 : L.ncol0;
  const int m = lb * kSegCols + lane;
  const bool valid = m < ncol;
  const int mm = valid ? m : ncol - 1;  // in-bounds column for loads of idle lanes
  const int nz = L.nz, Ls = seg_len(nz, NSEG);
  const int k0 = min(sg * Ls, nz), k1 = min(k0 + Ls, nz), len = k1 - k0;
  int i, j;
  col_ij(L, c, mm, i, j);
  const Nbr nb = ZERO ? Nbr{0, 0, 0, 0} : neighbours(L, i, j);
  const long long H = L.S;
  const TB *__restrict__ bb = bo + mm;
  const R *__restrict__ uw = uo + nb.w;
  const R *__restrict__ ue = uo + nb.e;
  const R *__restrict__ us = uo + nb.s;
  const R *__restrict__ un = uo + nb.n;
  R *__restrict__ ow = own + mm;
  const R *__restrict__ tx = tab + TX * L.P;
  const R *__restrict__ ty = tab + TY * L.P;
  const R *__restrict__ tz = tab + TZ * L.P;
  const R *__restrict__ ip = tab + TIP * L.P;
  const R *__restrict__ cf = tab + TCF * L.P;
  const R *__restrict__ pf = tab + TPF * L.P;
  const R *__restrict__ qb = tab + TQB * L.P;

  R y[SEG];
  R prev = R(0);
  // go: an update is pending (always in a single grid's step; a batched
  // grid's first step has none and sweeps with b = r as it is)
  double alpha = 0.0, rr = 0.0;
  bool go = false;
  if constexpr (UPD) {
    go = st->pending != 0;
    alpha = st->alpha;
  }
  if constexpr (ZERO && !UPD) {
    // no neighbour terms: every level's b is loaded first (levels past the
    // segment's end repeat its last one and are discarded), then the forward
    // recurrence runs in place, so no load waits behind a level's arithmetic
#pragma unroll
    for (int t = 0; t < SEG; ++t) y[t] = (R)ld_s<FINE>(&bb[(long long)min(k0 + t, k1 - 1) * H]);
#pragma unroll
    for (int t = 0; t < SEG; ++t) {
      if (t < len) {
        const int k = k0 + t;
        prev = (y[t] + tz[k] * prev) * ip[k];
        y[t] = prev;
      }
    }
  } else {
#pragma unroll
    for (int c0 = 0; c0 < SEG; c0 += 8) {
      if (c0 < len) {
        R g[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int k = min(k0 + c0 + t, k1 - 1);
          const long long o = (long long)k * H;
          R v;
          if constexpr (UPD) {
            // the residual update of the CG step; only the lane that owns the
            // column writes it (idle lanes, also those of blocks past the last
            // column, read it and must not see their own write)
            const double b0 = __builtin_nontemporal_load(&bb[o]);
            const double q0 = __builtin_nontemporal_load(&qo[mm + o]);
            const double rv = go ? b0 - alpha * q0 : b0;  // a select: q may hold anything without go
            if (go && valid && c0 + t < len) {
              __builtin_nontemporal_store(rv, &rw[mm + o]);
              rr += rv * rv;
            }
            v = (R)rv;
          } else {
            v = (R)ld_s<FINE>(&bb[o]);
          }
          if (!ZERO) {
            v = v + tx[k] * (uw[o] + ue[o]);
            v = v + ty[k] * (us[o] + un[o]);
          }
          g[t] = v;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (c0 + t < len) {
            const int k = k0 + c0 + t;
            prev = (g[t] + tz[k] * prev) * ip[k];
            y[c0 + t] = prev;
          }
        }
      }
    }
  }
  seg_join_store<R, ZERO, RHO1, FINE, SEG, NSEG>(y, prev, xch, sg, lane, k0, k1, len, nz, Ls, pf, cf, qb, valid, ow,
                                                 H, rho);
  if constexpr (UPD) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rr += __shfl_down(rr, o, 64);
    if (lane == 0) red[sg] = rr;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = 0.0;
      for (int w = 0; w < NSEG; ++w) v += red[w];
      partial[pbase + lb] = v;
    }
  }
}

// -------------------------------------------------------------------------
// Line relaxation with horizontally varying vertical coefficients (FP64,
// rho = 1, both horizontal directions), each column split into NSEG
// k-segments, one wavefront per segment.  Every column has its own factors,
// known per cell (tz3 = T_{k-1/2}, ip3 = 1/p_k, cf3 = T_{k+1/2}/p_k in the
// level's split layout), so the two recurrences of a segment run from zero and
// carry running products of their own multipliers, which the joins use where
// smooth_seg_body takes the shared per-level tables:
//   forward  y_k = (g_k + T_{k-1/2} y_{k-1}) / p_k,  pf_k = prod_{i=k0..k} T_{i-1/2}/p_i
//   backward w_k = y_k + (T_{k+1/2}/p_k) w_{k+1},    qb_k = prod_{i=k..k1-1} T_{i+1/2}/p_i
// y_k = y_k(local) + pf_k y_in, w_k = w_k(local) + qb_k w_in, with y_in / w_in
// the true values below / above the segment passed through LDS (an empty
// segment passes the identity).  Both arrays stay in registers (SEG >= the
// segment length); CH levels are loaded together (fewer with sixteen
// segments, whose 1024-lane blocks leave 128 registers per lane).  bo, uo,
// own: b of colour c, u of the other colour, u of colour c.
// -------------------------------------------------------------------------
// R: arithmetic and element type of u and tab; TB: element type of b (the
// FP32 preconditioner's finest level reads the FP64 CG residual); F: element
// type of the per-column fields (FP32 copies for the FP32 sweeps of the
// mixed-precision V-cycle).
// The finest level's fused CG forms, as in smooth_seg_body and the tiled
// sweeps: UPD (the first pre-smoothing pair, TB = double) advances b to
// b - alpha q, writes it back to rw and leaves the block's sum of its squares
// in partial[pbase + block]; DOT = 1 (the last post-smoothing pair) leaves
// <b, w> of the written columns there, DOT = 2 also <q, w> (qo: this colour's
// part of q), at partial[2 (pbase + block)] and [2 (pbase + block) + 1].
template <typename R, typename TB, typename F, bool ZERO, bool FINE, int SEG, int NSEG, int CH, int DOT = 0,
          bool UPD = false>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_seg3(Geo L, const R *__restrict__ tab, int c,
                                                           const TB *__restrict__ bo,
                                                           const R *__restrict__ uo,
                                                           R *__restrict__ own,
                                                           const int *__restrict__ done,
                                                           const F *__restrict__ tz3,
                                                           const F *__restrict__ ip3,
                                                           const F *__restrict__ cf3,
                                                           double *__restrict__ partial = nullptr, int pbase = 0,
                                                           double *__restrict__ rw = nullptr,
                                                           const double *__restrict__ qo = nullptr,
                                                           const PcgState *__restrict__ st = nullptr) {
  static_assert(!UPD || std::is_same<TB, double>::value, "the residual update reads the FP64 residual");
  static_assert(!(UPD && DOT), "one fused form per sweep");
  constexpr int NQ = DOT ? DOT : (UPD ? 1 : 0);
  __shared__ R xv[NSEG][kSegCols], xq[NSEG][kSegCols];
  __shared__ double red[NQ ? NSEG : 1][2];
  // DOT: each lane keeps its column's b in LDS for <b, w> (read again from
  // memory at the end, it would come back from HBM)
  __shared__ double bsh[DOT ? NSEG : 1][DOT ? SEG : 1][DOT ? kSegCols : 1];
  if (is_done(done)) return;
  const int lane = threadIdx.x & 63;
  const int sg = wave_id();
  const int ncol = c ? L.ncol1 : L.ncol0;
  const int m = logical_block() * kSegCols + lane;
  const bool valid = m < ncol;
  const int mm = valid ? m : ncol - 1;  // in-bounds column for the loads of idle lanes
  const int nz = L.nz, Ls = seg_len(nz, NSEG);
  const int k0 = min(sg * Ls, nz), k1 = min(k0 + Ls, nz), len = k1 - k0;
  int i, j;
  col_ij(L, c, mm, i, j);
  const Nbr nb = ZERO ? Nbr{0, 0, 0, 0} : neighbours(L, i, j);
  const long long H = L.S;
  const long long oc = (long long)c * L.cs + mm;
  const TB *__restrict__ bb = bo + mm;
  const R *__restrict__ uw = uo + nb.w;
  const R *__restrict__ ue = uo + nb.e;
  const R *__restrict__ us = uo + nb.s;
  const R *__restrict__ un = uo + nb.n;
  R *__restrict__ ow = own + mm;
  const F *__restrict__ zc = tz3 + oc;
  const F *__restrict__ pc = ip3 + oc;
  const F *__restrict__ fc = cf3 + oc;
  const R *__restrict__ tx = tab + TX * L.P;
  const R *__restrict__ ty = tab + TY * L.P;

  static_assert(SEG % CH == 0, "chunks must tile the segment");
  R y[SEG], pr[SEG];
  R prev = R(0), prod = R(1);
  // UPD: go, an update is pending (always in a single grid's step)
  double alpha = 0.0, rr = 0.0;
  bool go = false;
  if constexpr (UPD) {
    go = st->pending != 0;
    alpha = st->alpha;
  }
#pragma unroll
  for (int c0 = 0; c0 < SEG; c0 += CH) {
    if (c0 < len) {
      R g[CH], a[CH], d[CH];
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int k = min(k0 + c0 + t, k1 - 1);
        const long long o = (long long)k * H;
        R v;
        if constexpr (UPD) {
          // the residual update of the CG step; only the lane that owns the
          // column writes it
          const double b0 = __builtin_nontemporal_load(&bb[o]);
          const double q0 = __builtin_nontemporal_load(&qo[mm + o]);
          const double rv = go ? b0 - alpha * q0 : b0;  // a select: q may hold anything without go
          if (go && valid && c0 + t < len) {
            __builtin_nontemporal_store(rv, &rw[mm + o]);
            rr += rv * rv;
          }
          v = (R)rv;
        } else {
          const TB braw = ld_s<FINE>(&bb[o]);
          v = (R)braw;
          if constexpr (DOT > 0) bsh[sg][c0 + t][lane] = (double)braw;
        }
        if (!ZERO) {
          v = v + tx[k] * (uw[o] + ue[o]);
          v = v + ty[k] * (us[o] + un[o]);
        }
        g[t] = v;
        a[t] = (R)zc[o];
        d[t] = (R)pc[o];
      }
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        if (c0 + t < len) {
          prev = (g[t] + a[t] * prev) * d[t];
          prod = prod * (a[t] * d[t]);
          y[c0 + t] = prev;
          pr[c0 + t] = prod;
        }
      }
    }
  }
  // forward join: y_in of segment sg from the segments below it
  xv[sg][lane] = prev;
  xq[sg][lane] = prod;
  __syncthreads();
  R yin = R(0);
#pragma unroll
  for (int q = 0; q < NSEG - 1; ++q) {
    const R cand = xv[q][lane] + xq[q][lane] * yin;
    yin = q < sg ? cand : yin;
  }
  __syncthreads();
  // true y, then the local backward recurrence and its product (in place)
  R nxt = R(0), qprod = R(1);
#pragma unroll
  for (int c0 = SEG - CH; c0 >= 0; c0 -= CH) {
    if (c0 < len) {
      R e[CH];
#pragma unroll
      for (int t = 0; t < CH; ++t) e[t] = (R)fc[(long long)min(k0 + c0 + t, k1 - 1) * H];
#pragma unroll
      for (int t = CH - 1; t >= 0; --t) {
        if (c0 + t < len) {
          const R yt = y[c0 + t] + pr[c0 + t] * yin;
          nxt = yt + e[t] * nxt;
          qprod = qprod * e[t];
          y[c0 + t] = nxt;
          pr[c0 + t] = qprod;
        }
      }
    }
  }
  xv[sg][lane] = nxt;
  xq[sg][lane] = qprod;
  __syncthreads();
  R win = R(0);
#pragma unroll
  for (int q = NSEG - 1; q > 0; --q) {
    const R cand = xv[q][lane] + xq[q][lane] * win;
    win = q > sg ? cand : win;
  }
  double d0 = 0.0, d1 = 0.0;  // DOT: <b, w>, <q, w> of this lane's column
  if (valid) {
#pragma unroll
    for (int t = 0; t < SEG; ++t)
      if (t < len) {
        const long long o = (long long)(k0 + t) * H;
        const R w = y[t] + pr[t] * win;
        ow[o] = w;
        if constexpr (DOT > 0) {
          d0 += bsh[sg][t][lane] * (double)w;
          if constexpr (DOT == 2) d1 += __builtin_nontemporal_load(&qo[mm + o]) * (double)w;
        }
      }
  }
  if constexpr (NQ > 0) {
    double v0 = UPD ? rr : d0, v1 = d1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      v0 += __shfl_down(v0, o, 64);
      if constexpr (NQ == 2) v1 += __shfl_down(v1, o, 64);
    }
    if (lane == 0) {
      red[sg][0] = v0;
      red[sg][1] = v1;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
      double v = 0.0;
      for (int w = 0; w < NSEG; ++w) v += red[w][threadIdx.x];
      partial[(long long)(pbase + logical_block()) * NQ + threadIdx.x] = v;
    }
  }
}

// -------------------------------------------------------------------------
// One sweep pair of the coarsest level (colour 0, then colour 1, rho = 1;
// Alg. "Multigrid V-cycle", coarsest-level smoothing) in one launch.  A block
// owns an 8 x 8 tile of columns.  Phase A sweeps colour 0 on the tile and the
// ring of columns around it (50 columns, lane = column), from the old colour-1
// values; the ring's columns belong to neighbouring tiles, which compute the
// same values from the same operands, so the block needs nothing from them.
// The results go to LDS (and, for the tile's own columns, to memory).  Phase
// B sweeps the tile's 32 colour-1 columns with their colour-0 neighbours from
// LDS.  Both phases take the segmented column solve of smooth_seg_body and
// the tiled sweep (the same segments, recurrences, joins and operand order),
// so the result equals two half-sweep launches bitwise, with one launch
// boundary instead of two.  ZERO: the first pair of a V-cycle's coarsest
// solve, from u = 0 (phase A then has no neighbour terms).  Needs nx and ny
// multiples of 8, both horizontal directions, nz <= SEG * NSEG.
// Region coordinates (a, b) are relative to the tile's corner (i0, j0), both
// multiples of 8, so a column (a, b) has colour (a + b) & 1:
//   phase A lane l < 50: b = l / 5 - 1, a = (b odd ? -1 : 0) + 2 (l % 5)
//   phase B lane l < 32: b = l / 4,     a = (b odd ? 0 : 1) + 2 (l % 4)
// -------------------------------------------------------------------------
__device__ __forceinline__ int pair_lane_a(int a, int b) { return (b + 1) * 5 + ((a - ((b & 1) ? -1 : 0)) >> 1); }

template <typename R, bool ZERO, int SEG, int NSEG>
__global__ __launch_bounds__(NSEG * 64) void k_coarse_pair(Geo L, const R *__restrict__ tab,
                                                           const R *__restrict__ b, R *__restrict__ u,
                                                           const int *__restrict__ done) {
  __shared__ R xch[NSEG][kSegCols];
  __shared__ R cu[SEG * NSEG][kSegCols];  // phase A's colour-0 values: [level][lane]
  if (is_done(done)) return;
  const int tiles_x = L.nx >> 3, lb = logical_block();
  if (lb >= tiles_x * (L.ny >> 3)) return;  // whole blocks: no barrier is skipped
  const int lane = threadIdx.x & 63;
  const int sg = wave_id();
  const int i0 = (lb % tiles_x) << 3, j0 = (lb / tiles_x) << 3;
  const int nz = L.nz, Ls = seg_len(nz, NSEG);
  const int k0 = min(sg * Ls, nz), k1 = min(k0 + Ls, nz), len = k1 - k0;
  const long long H = L.S, cs = L.cs;
  const R *__restrict__ tx = tab + TX * L.P;
  const R *__restrict__ ty = tab + TY * L.P;
  const R *__restrict__ tz = tab + TZ * L.P;
  const R *__restrict__ ip = tab + TIP * L.P;
  const R *__restrict__ cf = tab + TCF * L.P;
  const R *__restrict__ pf = tab + TPF * L.P;
  const R *__restrict__ qb = tab + TQB * L.P;

  // ---- phase A: colour 0 on the tile and its ring
  {
    const bool valid = lane < 50;
    const int l = valid ? lane : 0;
    const int bb = l / 5 - 1, aa = ((bb & 1) ? -1 : 0) + 2 * (l % 5);
    const int i = wrapi(i0 + aa, L.nx), j = wrapi(j0 + bb, L.ny);
    const long long m = col_m(L, i, j);
    const Nbr nb = neighbours(L, i, j);
    const R *__restrict__ b0 = b + m;
    const R *__restrict__ u1 = u + cs;
    R y[SEG];
    R prev = R(0);
#pragma unroll
    for (int c0 = 0; c0 < SEG; c0 += 8) {
      if (c0 < len) {
        R g[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int k = min(k0 + c0 + t, k1 - 1);
          const long long o = (long long)k * H;
          R v = b0[o];
          if (!ZERO) {
            v = v + tx[k] * (u1[nb.w + o] + u1[nb.e + o]);
            v = v + ty[k] * (u1[nb.s + o] + u1[nb.n + o]);
          }
          g[t] = v;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (c0 + t < len) {
            const int k = k0 + c0 + t;
            prev = (g[t] + tz[k] * prev) * ip[k];
            y[c0 + t] = prev;
          }
        }
      }
    }
    seg_join_store<R, ZERO, true, false, SEG, NSEG>(y, prev, xch, sg, lane, k0, k1, len, nz, Ls, pf, cf, qb, valid,
                                                    &cu[0][lane], kSegCols, R(1));
    // the tile's own columns to memory (this lane wrote them: no barrier)
    if (valid && aa >= 0 && aa < 8 && bb >= 0 && bb < 8) {
      R *__restrict__ ow = u + m;
      for (int k = k0; k < k1; ++k) ow[(long long)k * H] = cu[k][lane];
    }
  }
  __syncthreads();
  // ---- phase B: colour 1 on the tile
  {
    const bool valid = lane < 32;
    const int l = valid ? lane : 0;
    const int bb = l >> 2, aa = ((bb & 1) ? 0 : 1) + 2 * (l & 3);
    const long long m = col_m(L, i0 + aa, j0 + bb);
    const int lw = pair_lane_a(aa - 1, bb), le = pair_lane_a(aa + 1, bb);
    const int ls = pair_lane_a(aa, bb - 1), ln = pair_lane_a(aa, bb + 1);
    const R *__restrict__ b1 = b + cs + m;
    R y[SEG];
    R prev = R(0);
#pragma unroll
    for (int c0 = 0; c0 < SEG; c0 += 8) {
      if (c0 < len) {
        R g[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int k = min(k0 + c0 + t, k1 - 1);
          R v = b1[(long long)k * H];
          v = v + tx[k] * (cu[k][lw] + cu[k][le]);
          v = v + ty[k] * (cu[k][ls] + cu[k][ln]);
          g[t] = v;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (c0 + t < len) {
            const int k = k0 + c0 + t;
            prev = (g[t] + tz[k] * prev) * ip[k];
            y[c0 + t] = prev;
          }
        }
      }
    }
    seg_join_store<R, false, true, false, SEG, NSEG>(y, prev, xch, sg, lane, k0, k1, len, nz, Ls, pf, cf, qb, valid,
                                                     u + cs + m, H, R(1));
  }
}

// -------------------------------------------------------------------------
// The same FP64 half-sweep with rho = 1 after the first sweep, with the other
// colour staged in LDS (FINE: the finest level, streaming accesses).  Five
// 64-lane loads per level (b and four neighbours) keep the texture units near
// saturation although the neighbours hit in cache; here a block owns 64
// columns of colour c arranged as 32 m-columns by 2 rows, one k-segment per
// wavefront, and per level a wavefront loads its b (8 bytes per lane), the
// other colour's 4 x 32 interior values of rows j0-1 .. j0+2 (16 bytes per
// lane) and the two wrapped end values its own rows read (2 lanes), stages
// them in its own LDS slot and reads the four neighbours there.  Needs nx/2
// even (16-byte aligned pairs) and ny even.  LDS slot layout per row: [1]
// left end, [2 + x] interior x, [2 + nxm] right end (interior pairs start at
// even indices, so pair writes are aligned).
// -------------------------------------------------------------------------
constexpr int kSTX = 32;  // m-columns per tile
constexpr int kCRow = 48;  // LDS row stride of the staged coarse values (40 used)

// DOT = 1 (the last two half-sweeps of a preconditioner application): also
// the block's partial sum of <b, w> over its written columns, into
// partial[pbase + lb]; DOT = 2: <b, w> and <q, w> (q: the colour's part of
// the CG vector q) into partial[2 (pbase + lb)] and [2 (pbase + lb) + 1].  The
// wavefront keeps its b values in LDS for that; a block's sum adds its
// wavefronts' sums in segment order.
// UPD (the first pre-smoothing pair, as in smooth_seg_body): b is advanced to
// b - alpha q and written back to rwc (this colour's CG residual), and the
// block's partial sum of its squares goes to partial[pbase + lb].
// PRO (colour 1, the first post-smoothing sweep, rho = 1): the colour-0
// values it reads are the V-cycle's values before the coarse correction (uo)
// and each staged one is corrected on the fly with the bilinear interpolation
// of the coarser level's correction uc (coarse geometry C), in the order of
// the column prolongation, so the correction is never written: the colour-0
// sweep that follows overwrites colour 0 without reading it.  The 3 x 36
// coarse values a wavefront's tile needs per level (rows J0-1 .. J0+1,
// columns mx0-2 .. mx0+33) are staged in LDS with two loads, even and odd
// columns apart.
// DOT = 3 (colour 0, the last sweep, classic beta, after a PRO sweep): <b, w>
// of the written columns plus <r1, z1> over the colour-1 cells of the tile's
// rows, z1 from the staged values and r1 loaded (r1c: colour 1 of r), into
// partial[pbase + lb].
// DOT = 4 (the same with the flexible beta): <b, w> + <r1, z1> and <q, w> +
// <q1, z1> (q1c: colour 1 of q) into partial[2 (pbase + lb)] and [... + 1].
// PAIR (with PRO; the coarse level's half-width, colour stride and plane
// stride even, its array 16-byte aligned): the staged coarse values come in
// pairs of neighbouring same-colour columns, one 16-byte load per lane on 60
// lanes instead of two 8-byte loads on 128.
// TU (with PRO): element type of uo and uc.  TU = float is the mixed-precision
// V-cycle's finest level: FP32 colour-0 values and FP32 coarse correction,
// the correction formed in FP32 and both widened before their FP64 sum, as in
// k_prolong_out_tile; the staged coarse values (128 floats per wavefront, row
// stride 40) then live in the wavefront's own row of the join exchange array,
// which the wavefront alone touches until the first join (a DOT sweep's LDS
// stays under half of a compute unit's).
// R: element type of the level (b, u, coefficients, arithmetic): float on
// the mixed-precision V-cycle's coarse levels (plain sweeps and PRO only).
template <int SEG, int NSEG, bool FINE, int DOT = 0, bool UPD = false, bool PRO = false, int CH = 8,
          bool PAIR = false, typename TU = double, typename R = double>
__device__ __forceinline__ void smooth_tile_body(Geo L, const R *__restrict__ tab, int c,
                                                 const R *__restrict__ bo,
                                                 const TU *__restrict__ uo,
                                                 R *__restrict__ own,
                                                 const int *__restrict__ done, int lb,
                                                 double *__restrict__ partial = nullptr, int pbase = 0,
                                                 const double *__restrict__ qc = nullptr,
                                                 double *__restrict__ rwc = nullptr,
                                                 const PcgState *__restrict__ st = nullptr,
                                                 const Geo *Cg = nullptr,
                                                 const typename std::common_type<TU>::type *__restrict__ uc = nullptr,
                                                 const double *__restrict__ r1c = nullptr,
                                                 const double *__restrict__ q1c = nullptr) {
  constexpr bool F32 = std::is_same<TU, float>::value;
  constexpr bool ALIAS = F32 && std::is_same<R, double>::value;  // staged coarse values in xch rows
  static_assert(std::is_same<TU, R>::value || PRO, "mixed element types only with the fused prolongation");
  static_assert(std::is_same<R, double>::value || (DOT == 0 && !UPD), "CG forms only on FP64 levels");
  typedef TU nt_p2 __attribute__((ext_vector_type(2)));  // a pair of staged values
  typedef R nt_r2 __attribute__((ext_vector_type(2)));   // a pair of level values
  constexpr int CR = F32 ? 40 : kCRow;                      // row stride of the staged coarse values
  constexpr int NQ = DOT ? (DOT == 3 ? 1 : (DOT == 4 ? 2 : DOT)) : (UPD ? 1 : 0);  // partial sums per block
  constexpr int SJ = DOT == 3 ? 1 : (DOT == 4 ? 2 : DOT);                         // seg_join_store's products
  if constexpr (UPD) {
    // no update pending (a batched grid's first step): the plain sweep of b = r
    if (st->pending == 0) {
      smooth_tile_body<SEG, NSEG, FINE, 0, false, false, CH>(L, tab, c, bo, uo, own, done, lb);
      return;
    }
  }
  __shared__ R xch[NSEG][kSegCols];
  __shared__ __align__(16) R ot[NSEG][4][36];
  __shared__ double bsh[DOT ? NSEG : 1][DOT ? SEG : 1][64];
  __shared__ double red[NQ ? NSEG : 1][2];
  __shared__ __align__(16) TU csl[PRO && !ALIAS ? NSEG : 1][PRO && !ALIAS ? (F32 ? 128 : 3 * kCRow) : 1];
  const int tiles_x = (L.hx2 + kSTX - 1) / kSTX;
  if (is_done(done) || lb >= tiles_x * (L.ny / 2)) return;  // whole blocks: no barrier is skipped
  const int lane = threadIdx.x & 63;
  const int sg = wave_id();
  const int ty = lb / tiles_x, tx = lb - ty * tiles_x;
  const int mx0 = tx * kSTX, j0 = ty * 2;
  const int nxm = min(kSTX, L.hx2 - mx0);
  const int x = lane & 31, r = lane >> 5;
  const int j = j0 + r;
  const bool valid = x < nxm;
  const int xm = valid ? x : nxm - 1;
  const long long mo = (long long)j * L.hx2 + mx0 + xm;  // own split column
  const int par = (j + c) & 1;                            // 1: the own cell sits at an odd i
  // staging: interior pair of this lane, end value of lanes 0..7
  const int rr = lane >> 4, pp = lane & 15;
  const bool pv = 2 * pp < nxm;
  const long long po = (long long)wrapi(j0 - 1 + rr, L.ny) * L.hx2 + mx0 + (pv ? 2 * pp : 0);
  // end values: lane 0 for own row j0 (slot row 1), lane 1 for j0 + 1 (slot
  // row 2), each the one side its parity reads (left end: even, right: odd)
  const int er = 1 + (lane & 1), side = (j0 + (lane & 1) + c) & 1;
  const long long eo = (long long)(j0 - 1 + er) * L.hx2 + (side ? (mx0 + nxm) % L.hx2 : (mx0 - 1 + L.hx2) % L.hx2);
  const int ei = side ? nxm + 2 : 1;
  const long long H = L.S;
  const int nz = L.nz, Ls = seg_len(nz, NSEG);
  const int k0 = min(sg * Ls, nz), k1 = min(k0 + Ls, nz), len = k1 - k0;
  const R *__restrict__ txv = tab + TX * L.P;
  const R *__restrict__ tyv = tab + TY * L.P;
  const R *__restrict__ tz = tab + TZ * L.P;
  const R *__restrict__ ip = tab + TIP * L.P;
  const R *__restrict__ cf = tab + TCF * L.P;
  const R *__restrict__ pf = tab + TPF * L.P;
  const R *__restrict__ qb = tab + TQB * L.P;
  R(*slot)[36] = ot[sg];
  const TU *ug = gp(uo);
  const R *bg = gp(bo);
  const double *qg = UPD ? gp(qc) : nullptr;
  double alpha = 0.0, rsq = 0.0;
  if constexpr (UPD) alpha = st->alpha;
  // PRO: this lane's two coarse staging values and their LDS slots, and its
  // corrections' rows.  Staging value v < 120 is coarse row J0 - 1 + v / 40,
  // column I = mx0 - 4 + 2 t + par (rem = v % 40 = 20 par + t), at slot
  // row * kCRow + rem: the even columns of a row, then the odd ones, so the
  // neighbours a lane reads lie 8 bytes apart across lanes (interleaved they
  // were 16 bytes apart, a two-way LDS bank conflict on every read); values
  // no staged fine cell reads, and v >= 120, load an in-bounds dummy.
  long long co0 = 0, co1 = 0, HC = 0;
  int cs0 = 0, cs1 = 0;
  const TU *ucg = nullptr;
  TU *csf = nullptr;
  int pa = 0, pb = 0, pd = 0, ea = 0, eb = 0, ed = 0;
  if constexpr (PRO) {
    const Geo C = *Cg;
    const int J0 = j0 >> 1;
    auto coff = [&](int v) -> long long {
      const int row = v / 40, rem = v - row * 40, par = rem / 20, t = rem - par * 20;
      const int q = 2 * t + par - 2;  // I - (mx0 - 2)
      const bool need = v < 120 && q >= 0 && q <= nxm + 3;
      const int I = wrapi(mx0 - 2 + (need ? q : 0), C.nx);
      const int J = wrapi(J0 - 1 + (need ? row : 0), C.ny);
      return (long long)((I + J) & 1) * C.cs + col_m(C, I, J);
    };
    auto cslot = [](int v) -> int { return v < 120 ? (v / 40) * CR + v % 40 : 2 * CR + 40 + (v - 120); };
    if constexpr (PAIR) {
      // lane v < 60: row v / 20, parity par = (v % 20) / 10, pair t2 = v % 10,
      // columns I = mx0 - 4 + 4 t2 + par and I + 2 (split neighbours: with the
      // half-width even, I - par is a multiple of 4 also after the wrap, so a
      // pair starts at an even split index and never straddles the wrap);
      // pairs no staged fine cell reads, and v >= 60, load an aligned dummy
      const int v = lane, row = v / 20, rem = v - row * 20, par = rem / 10, t2 = rem - par * 10;
      const int q = 4 * t2 + par - 2;  // I - (mx0 - 2) of the pair's first column
      const bool need = v < 60 && q + 2 >= 0 && q <= nxm + 3;
      const int I = wrapi(mx0 - 2 + (need ? q : 2), C.nx);
      const int J = wrapi(J0 - 1 + (need ? row : 1), C.ny);
      co0 = (long long)((I + J) & 1) * C.cs + col_m(C, I, J);
      cs0 = v < 60 ? row * CR + par * 20 + 2 * t2 : 2 * CR + 40 + 2 * (v - 60);
    } else {
      co0 = coff(lane);
      co1 = coff(64 + lane);
      cs0 = cslot(lane);
      cs1 = cslot(64 + lane);
    }
    HC = C.S;
    ucg = gp(uc);
    if constexpr (ALIAS) csf = reinterpret_cast<TU *>(&xch[sg][0]);
    else csf = csl[sg];
    // staged row q -> coarse rows of its parent (pa) and y-neighbour (pb),
    // x-neighbour direction pd (fine row odd: +1)
    pa = (rr + 1) >> 1;
    pb = (rr & 1) ? pa - 1 : pa + 1;
    pd = (rr & 1) ? -1 : 1;
    ea = (er + 1) >> 1;
    eb = (er & 1) ? ea - 1 : ea + 1;
    ed = (er & 1) ? -1 : 1;
  }
  // the bilinear correction of the staged colour-0 value at index idx of a
  // staged row (coarse rows a, b, direction d; coarse column I = mx0 - 2 + q
  // sits at slot row * kCRow + 20 ((q + 2) & 1) + ((q + 2) >> 1)), in the
  // column kernel's order
  auto cv = [&](int row, int q) -> TU { return csf[row * CR + 20 * ((q + 2) & 1) + ((q + 2) >> 1)]; };
  auto corr = [&](int a, int b, int d, int idx) -> TU {
    TU e = TU(9.0 / 16.0) * cv(a, idx);
    e = e + TU(3.0 / 16.0) * cv(a, idx + d);
    e = e + TU(3.0 / 16.0) * cv(b, idx);
    e = e + TU(1.0 / 16.0) * cv(b, idx + d);
    return e;
  };
  const double *r1g = DOT >= 3 ? gp(r1c) : nullptr;
  const double *q1g = DOT == 4 ? gp(q1c) : nullptr;
  double d1 = 0.0, d2 = 0.0;  // DOT 3, 4: <r1, z1> (and <q1, z1>) of this lane's colour-1 cell

  R y[SEG];
  R prev = R(0);
#pragma unroll
  for (int c0 = 0; c0 < SEG; c0 += CH) {
    if (c0 < len) {
      R bv[CH];
      double qv[UPD ? CH : 1], r1v[DOT >= 3 ? CH : 1], q1v[DOT == 4 ? CH : 1];
      TU ev[CH], cv0[PRO && !PAIR ? CH : 1], cv1[PRO && !PAIR ? CH : 1];
      nt_p2 cvp[PRO && PAIR ? CH : 1];
      nt_p2 tv[CH];
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int kc = min(k0 + c0 + t, k1 - 1);
        const long long o = (long long)kc * H;
        bv[t] = ld_s<FINE>(&bg[o + mo]);
        if constexpr (UPD) qv[t] = __builtin_nontemporal_load(&qg[o + mo]);
        tv[t] = *(const nt_p2 *)&ug[o + po];
        ev[t] = lane < 2 ? ug[o + eo] : TU(0);
        if constexpr (PRO) {
          if constexpr (PAIR) {
            cvp[t] = *(const nt_p2 *)&ucg[kc * HC + co0];
          } else {
            cv0[t] = ucg[kc * HC + co0];
            cv1[t] = ucg[kc * HC + co1];
          }
        }
        if constexpr (DOT >= 3) r1v[t] = __builtin_nontemporal_load(&r1g[o + mo]);
        if constexpr (DOT == 4) q1v[t] = __builtin_nontemporal_load(&q1g[o + mo]);
      }
      // Every level of the chunk runs without a branch (levels past the
      // segment's end repeat its last level and are discarded), so no load is
      // moved into a conditional block next to its first use.
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int k = min(k0 + c0 + t, k1 - 1);
        // stage level k (LDS operations of a wavefront complete in order; the
        // empty asm keeps the compiler from moving them across each other).
        // Lanes past the tile's last pair write pads or the right end's place,
        // which the end values written next overwrite.
        nt_r2 pr = {(R)tv[t].x, (R)tv[t].y};
        R evk = (R)ev[t];
        if constexpr (PRO) {
          if constexpr (PAIR) {
            *(nt_p2 *)&csf[cs0] = cvp[t];
          } else {
            csf[cs0] = cv0[t];
            csf[cs1] = cv1[t];
          }
          __asm__ volatile("" ::: "memory");
          // the pair's columns idx0 = 2 + 2 pp and idx0 + 1 read three coarse
          // values per row (columns idx0, idx0 + 1 and idx0 + 2 or idx0 - 1):
          // slots base, base + 20 and base + 1 or base + 19
          const int sa = pa * CR + 2 + pp, sb = pb * CR + 2 + pp, s2 = pd > 0 ? 1 : 19;
          const TU a0 = csf[sa], a1 = csf[sa + 20], a2 = csf[sa + s2];
          const TU b0 = csf[sb], b1 = csf[sb + 20], b2 = csf[sb + s2];
          TU e0 = TU(9.0 / 16.0) * a0;
          e0 = e0 + TU(3.0 / 16.0) * (pd > 0 ? a1 : a2);
          e0 = e0 + TU(3.0 / 16.0) * b0;
          e0 = e0 + TU(1.0 / 16.0) * (pd > 0 ? b1 : b2);
          TU e1 = TU(9.0 / 16.0) * a1;
          e1 = e1 + TU(3.0 / 16.0) * (pd > 0 ? a2 : a0);
          e1 = e1 + TU(3.0 / 16.0) * b1;
          e1 = e1 + TU(1.0 / 16.0) * (pd > 0 ? b2 : b0);
          pr.x = pr.x + (R)e0;
          pr.y = pr.y + (R)e1;
          if (lane < 2) evk = evk + (R)corr(ea, eb, ed, ei);
          __asm__ volatile("" ::: "memory");
        }
        *(nt_r2 *)&slot[rr][2 + 2 * pp] = pr;
        __asm__ volatile("" ::: "memory");
        if (lane < 2) slot[er][ei] = evk;
        __asm__ volatile("" ::: "memory");
        const R w = slot[r + 1][x + 1 + par], e = slot[r + 1][x + 2 + par];
        const R so = slot[r][x + 2], no = slot[r + 2][x + 2];
        if constexpr (DOT >= 3) {
          const double z1 = slot[r + 1][x + 2];  // the colour-1 cell (j, mx0 + x)
          const bool on = valid && c0 + t < len;
          d1 += on ? r1v[t] * z1 : 0.0;
          if constexpr (DOT == 4) d2 += on ? q1v[t] * z1 : 0.0;
        }
        __asm__ volatile("" ::: "memory");
        R g = bv[t];
        if constexpr (UPD) {
          // the residual update of the CG step; only the lane that owns the
          // column writes it
          g = bv[t] - alpha * qv[t];
          if (valid && c0 + t < len) {
            __builtin_nontemporal_store(g, &rwc[(long long)k * H + mo]);
            rsq += g * g;
          }
        }
        g = g + txv[k] * (w + e);
        g = g + tyv[k] * (so + no);
        const R nv = (g + tz[k] * prev) * ip[k];
        prev = c0 + t < len ? nv : prev;
        y[c0 + t] = prev;
        if constexpr (DOT > 0) bsh[sg][c0 + t][lane] = bv[t];
      }
    }
  }
  double dsum[2] = {UPD ? rsq : d1, d2};
  seg_join_store<R, false, true, FINE, SEG, NSEG, SJ>(y, prev, xch, sg, lane, k0, k1, len, nz, Ls, pf, cf,
                                                      qb, valid, own + mo, H, R(1), &bsh[DOT ? sg : 0][0][0],
                                                           (DOT == 2 || DOT == 4) ? qc + mo : nullptr, dsum);
  if constexpr (NQ > 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double v = dsum[q];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if (lane == 0) red[sg][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
      double v = 0.0;
      for (int w = 0; w < NSEG; ++w) v += red[w][threadIdx.x];
      partial[(long long)(pbase + lb) * NQ + threadIdx.x] = v;
    }
  }
}

template <int SEG, int NSEG, bool FINE, typename R = double>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_tile(Geo L, const R *__restrict__ tab, int c,
                                                           const R *__restrict__ bo,
                                                           const R *__restrict__ uo,
                                                           R *__restrict__ own,
                                                           const int *__restrict__ done) {
  smooth_tile_body<SEG, NSEG, FINE, 0, false, false, 8, false, R, R>(L, tab, c, bo, uo, own, done, logical_block());
}

// The finest level's colour-1 half-sweep of the first pre-smoothing pair
// with the CG residual update fused in.
template <int SEG, int NSEG>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_tile_upd(Geo L, const double *__restrict__ tab, int c,
                                                               double *__restrict__ rc,
                                                               const double *__restrict__ uo,
                                                               double *__restrict__ own,
                                                               const double *__restrict__ qc,
                                                               const PcgState *__restrict__ st,
                                                               double *__restrict__ partial, int pbase) {
  smooth_tile_body<SEG, NSEG, true, 0, true>(L, tab, c, rc, uo, own, &st->done, logical_block(), partial, pbase, qc,
                                             rc, st);
}

// A level's first post-smoothing sweep (colour 1) with the coarse correction
// of colour 0 applied on the fly (no separate prolongation); FINE: the finest
// level (streaming accesses).
template <int SEG, int NSEG, bool FINE = true, bool PAIR = false, typename R = double>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_tile_pro(Geo L, Geo C, const R *__restrict__ tab,
                                                               const R *__restrict__ bo,
                                                               const R *__restrict__ uo,
                                                               R *__restrict__ own,
                                                               const R *__restrict__ uc,
                                                               const int *__restrict__ done) {
  smooth_tile_body<SEG, NSEG, FINE, 0, false, true, 4, PAIR, R, R>(L, tab, 1, bo, uo, own, done, logical_block(),
                                                                   nullptr, 0, nullptr, nullptr, nullptr, &C, uc);
}

// The mixed-precision V-cycle's finest colour-1 post-smoothing sweep (FP64)
// with the last prolongation applied on the fly: it reads the FP32 colour-0
// values of the pre-smoothed iterate and the FP32 coarse correction, and the
// colour-0 values it stages are the ones the prolongation pass would write
// into the FP64 output (base + P e, e in FP32, the sum in FP64); DOT as
// k_smooth_tile_dot.
template <int SEG, int NSEG, int DOT, bool PAIR>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_tile_pro32(Geo L, Geo C, const double *__restrict__ tab,
                                                                 const double *__restrict__ bo,
                                                                 const float *__restrict__ uo,
                                                                 double *__restrict__ own,
                                                                 const float *__restrict__ uc,
                                                                 const int *__restrict__ done,
                                                                 double *__restrict__ partial, int pbase,
                                                                 const double *__restrict__ qc) {
  smooth_tile_body<SEG, NSEG, true, DOT, false, true, 4, PAIR, float>(L, tab, 1, bo, uo, own, done, logical_block(),
                                                                      partial, pbase, qc, nullptr, nullptr, &C, uc);
}

// The last sweep (colour 0) after it, with <r, z> of both colours.
template <int SEG, int NSEG>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_tile_dot3(Geo L, const double *__restrict__ tab,
                                                                const double *__restrict__ bo,
                                                                const double *__restrict__ uo,
                                                                double *__restrict__ own,
                                                                const int *__restrict__ done,
                                                                double *__restrict__ partial,
                                                                const double *__restrict__ r1c) {
  smooth_tile_body<SEG, NSEG, true, 3, false, false, 4>(L, tab, 0, bo, uo, own, done, logical_block(), partial, 0,
                                                        nullptr, nullptr, nullptr, nullptr, nullptr, r1c);
}

// The same with the flexible beta: <r, z> and <z, q> of both colours.
template <int SEG, int NSEG>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_tile_dot4(Geo L, const double *__restrict__ tab,
                                                                const double *__restrict__ bo,
                                                                const double *__restrict__ uo,
                                                                double *__restrict__ own,
                                                                const int *__restrict__ done,
                                                                double *__restrict__ partial,
                                                                const double *__restrict__ r1c,
                                                                const double *__restrict__ q0c,
                                                                const double *__restrict__ q1c) {
  smooth_tile_body<SEG, NSEG, true, 4, false, false, 4>(L, tab, 0, bo, uo, own, done, logical_block(), partial, 0,
                                                        q0c, nullptr, nullptr, nullptr, nullptr, r1c, q1c);
}

// The finest level's tiled half-sweep with the fused CG inner products.
template <int SEG, int NSEG, int DOT>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_tile_dot(Geo L, const double *__restrict__ tab, int c,
                                                               const double *__restrict__ bo,
                                                               const double *__restrict__ uo,
                                                               double *__restrict__ own,
                                                               const int *__restrict__ done,
                                                               double *__restrict__ partial, int pbase,
                                                               const double *__restrict__ qc) {
  smooth_tile_body<SEG, NSEG, true, DOT>(L, tab, c, bo, uo, own, done, logical_block(), partial, pbase, qc);
}

template <typename R, bool ZERO, bool RHO1, bool FINE, int SEG, int NSEG, typename TB = R>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_seg(Geo L, const R *__restrict__ tab, int c,
                                                          const TB *__restrict__ bo,
                                                          const R *__restrict__ uo,
                                                          R *__restrict__ own, R rho,
                                                          const int *__restrict__ done) {
  smooth_seg_body<R, ZERO, RHO1, FINE, SEG, NSEG, TB>(L, tab, c, bo, uo, own, rho, done, logical_block(), gridDim.x);
}

// The finest level's first pre-smoothing pair with the CG residual update
// fused in (column kernel; rho = 1).
template <typename R, bool ZERO, int SEG, int NSEG>
__global__ __launch_bounds__(NSEG * 64) void k_smooth_seg_upd(Geo L, const R *__restrict__ tab, int c,
                                                              double *__restrict__ rc, const R *__restrict__ uo,
                                                              R *__restrict__ own, const double *__restrict__ qc,
                                                              const PcgState *__restrict__ st,
                                                              double *__restrict__ partial, int pbase) {
  smooth_seg_body<R, ZERO, true, true, SEG, NSEG, double, true>(L, tab, c, rc, uo, own, R(1), &st->done,
                                                                logical_block(), gridDim.x, rc, qc, st, partial,
                                                                pbase);
}

// Residual (b - A u) of one cell given its column neighbours at level k.
template <typename R>
__device__ __forceinline__ R cell_residual(R bk, R vk, R txk, R tyk, R tzlo, R tzhi, R uc, R um,
                                           R up, R uW, R uE, R uS, R uN, int hasx, int hasy) {
  R acc = vk * uc;
  if (hasx) {
    acc = acc + txk * (uc - uW);
    acc = acc + txk * (uc - uE);
  }
  if (hasy) {
    acc = acc + tyk * (uc - uS);
    acc = acc + tyk * (uc - uN);
  }
  acc = acc + tzlo * (uc - um);
  acc = acc + tzhi * (uc - up);
  return bk - acc;
}

// -------------------------------------------------------------------------
// Residual + restriction right after a colour-1 sweep with rho = 1: the
// colour-1 children have zero residual, so each coarse column needs only its
// two colour-0 children (2I, 2J) and (2I+1, 2J+1).  Their eight horizontal
// neighbours are six distinct colour-1 columns:
//   A = (2I-1, 2J)  B = (2I+1, 2J)  C = (2I, 2J-1)  D = (2I, 2J+1)
//   E = (2I+2, 2J+1)  F = (2I+1, 2J+2)
// child (2I,2J): W=A E=B S=C N=D;  child (2I+1,2J+1): W=D E=E S=B N=F.
// Requires both horizontal directions to have faces.  C3: the two children's
// vertical faces from the split-layout field tz3 (T_{k-1/2} at plane k; the
// top face is zero) instead of the table.
// -------------------------------------------------------------------------
template <typename R, typename TB = R, int NSEG = kSeg, bool C3 = false>
__device__ __forceinline__ void resid_restrict_bz_body(Geo F, Geo C,
                                                              const R *__restrict__ tab,
                                                              const TB *__restrict__ b,
                                                              const R *__restrict__ u,
                                                              R *__restrict__ bc,
                                                              const int *__restrict__ done, int lb, int nblocks,
                                                              const R *__restrict__ tz3 = nullptr) {
  constexpr int U = 4;
  if (is_done(done)) return;
  const int gid = lb * kSegCols + (threadIdx.x & 63);
  if (gid >= 2 * C.H) return;
  const int cc = gid & 1;  // lanes alternate coarse colours (adjacent coarse columns)
  const int mc = gid >> 1;
  if (mc >= (cc ? C.ncol1 : C.ncol0)) return;
  const int Ls = seg_len(F.nz, NSEG);
  const int k0 = min(wave_id() * Ls, F.nz), k1 = min(k0 + Ls, F.nz);
  int I, J;
  col_ij(C, cc, mc, I, J);
  const int i0 = 2 * I, j0 = 2 * J;
  const long long H = F.S;
  const R *__restrict__ ured = u;            // colour 0
  const R *__restrict__ ublk = u + F.cs;     // colour 1
  const R *__restrict__ u0 = ured + col_m(F, i0, j0);
  const R *__restrict__ u1 = ured + col_m(F, i0 + 1, j0 + 1);
  const TB *__restrict__ b0 = b + col_m(F, i0, j0);
  const TB *__restrict__ b1 = b + col_m(F, i0 + 1, j0 + 1);
  const R *__restrict__ pA = ublk + col_m(F, wrapi(i0 - 1, F.nx), j0);
  const R *__restrict__ pB = ublk + col_m(F, i0 + 1, j0);
  const R *__restrict__ pC = ublk + col_m(F, i0, wrapi(j0 - 1, F.ny));
  const R *__restrict__ pD = ublk + col_m(F, i0, j0 + 1);
  const R *__restrict__ pE = ublk + col_m(F, wrapi(i0 + 2, F.nx), j0 + 1);
  const R *__restrict__ pF = ublk + col_m(F, i0 + 1, wrapi(j0 + 2, F.ny));
  const R *__restrict__ tv = tab + TV * F.P;
  const R *__restrict__ tx = tab + TX * F.P;
  const R *__restrict__ ty = tab + TY * F.P;
  const R *__restrict__ tz = tab + TZ * F.P;
  R *__restrict__ out = bc + (long long)cc * C.cs + mc;
  const int nz = F.nz;
  if (k1 <= k0) return;
  // C3: the children's faces (both colour 0)
  const R *__restrict__ z0 = C3 ? tz3 + col_m(F, i0, j0) : nullptr;
  const R *__restrict__ z1 = C3 ? tz3 + col_m(F, i0 + 1, j0 + 1) : nullptr;
  R c0 = u0[(long long)k0 * H], c1 = u1[(long long)k0 * H];
  R m0 = k0 > 0 ? u0[(long long)(k0 - 1) * H] : c0;
  R m1 = k0 > 0 ? u1[(long long)(k0 - 1) * H] : c1;
  R f0 = R(0), f1 = R(0);  // C3: the faces below level k
  if constexpr (C3) {
    f0 = z0[(long long)k0 * H];
    f1 = z1[(long long)k0 * H];
  }
  auto step = [&](int k, R bb0, R bb1, R p0, R p1, R A, R B, R Cv, R D, R E, R Fv, R g0, R g1) {
    R lo0 = tz[k], hi0 = tz[k + 1], lo1 = tz[k], hi1 = tz[k + 1];
    if constexpr (C3) {
      lo0 = f0;
      lo1 = f1;
      hi0 = k + 1 < nz ? g0 : R(0);
      hi1 = k + 1 < nz ? g1 : R(0);
      f0 = g0;
      f1 = g1;
    }
    const R r0 = cell_residual<R>(bb0, tv[k], tx[k], ty[k], lo0, hi0, c0, m0, p0, A, B, Cv, D, 1, 1);
    const R r1 = cell_residual<R>(bb1, tv[k], tx[k], ty[k], lo1, hi1, c1, m1, p1, D, E, B, Fv, 1, 1);
    out[(long long)k * C.S] = r0 + r1;
    m0 = c0;
    c0 = p0;
    m1 = c1;
    c1 = p1;
  };
  int k = k0;
  for (; k + U <= k1; k += U) {
    R bb0[U], bb1[U], p0[U], p1[U], A[U], B[U], Cv[U], D[U], E[U], Fv[U], g0[U], g1[U];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const long long o = (long long)(k + t) * H;
      const long long op = (long long)min(k + t + 1, nz - 1) * H;
      bb0[t] = (R)b0[o];
      bb1[t] = (R)b1[o];
      p0[t] = u0[op];
      p1[t] = u1[op];
      A[t] = pA[o];
      B[t] = pB[o];
      Cv[t] = pC[o];
      D[t] = pD[o];
      E[t] = pE[o];
      Fv[t] = pF[o];
      if constexpr (C3) {  // the faces above level k + t (level k + t + 1's, clamped)
        g0[t] = z0[op];
        g1[t] = z1[op];
      } else {
        g0[t] = g1[t] = R(0);
      }
    }
#pragma unroll
    for (int t = 0; t < U; ++t)
      step(k + t, bb0[t], bb1[t], p0[t], p1[t], A[t], B[t], Cv[t], D[t], E[t], Fv[t], g0[t], g1[t]);
  }
  for (; k < k1; ++k) {
    const long long o = (long long)k * H;
    const long long op = (long long)min(k + 1, nz - 1) * H;
    step(k, (R)b0[o], (R)b1[o], u0[op], u1[op], pA[o], pB[o], pC[o], pD[o], pE[o], pF[o], C3 ? z0[op] : R(0),
         C3 ? z1[op] : R(0));
  }
}

// NSEG k-segments per column, one wavefront each (more on small coarse levels,
// where the sequential walk over a segment is the kernel's latency).
template <typename R, typename TB = R, int NSEG = kSeg, bool C3 = false>
__global__ __launch_bounds__(NSEG * 64) void k_resid_restrict_bz(Geo F, Geo C,
                                                                 const R *__restrict__ tab,
                                                                 const TB *__restrict__ b,
                                                                 const R *__restrict__ u,
                                                                 R *__restrict__ bc,
                                                                 const int *__restrict__ done,
                                                                 const R *__restrict__ tz3 = nullptr) {
  resid_restrict_bz_body<R, TB, NSEG, C3>(F, C, tab, b, u, bc, done, logical_block(), gridDim.x, tz3);
}

// -------------------------------------------------------------------------
// Residual on the fine level summed over 2x2 children into the coarse
// right-hand side (Alg. "Multigrid V-cycle": residual, then restriction).
// One lane per coarse column.  BZ: children of colour 1 carry a zero residual
// (they were just solved exactly), so only the two colour-0 children are
// evaluated.
// -------------------------------------------------------------------------
// C3: the vertical faces of each child column from the split-layout field
// tz3 (T_{k-1/2}) instead of the table.
// TB: element type of b (the mixed-precision V-cycle's finest level reads the
// FP64 CG residual).
template <typename R, bool BZ, bool C3 = false, typename TB = R>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(Geo F, Geo C, const R *__restrict__ tab,
                                                           const TB *__restrict__ b,
                                                           const R *__restrict__ u,
                                                           R *__restrict__ bc,
                                                           const int *__restrict__ done,
                                                           const R *__restrict__ tz3 = nullptr) {
  if (is_done(done)) return;
  const int gid = logical_block() * kBlock + threadIdx.x;
  if (gid >= 2 * C.H) return;
  const int cc = gid & 1;
  const int mc = gid >> 1;
  if (mc >= (cc ? C.ncol1 : C.ncol0)) return;
  int I, J;
  col_ij(C, cc, mc, I, J);

  // children in the order (0,0), (1,0), (0,1), (1,1); colour of (a,b) is (a+b)&1
  constexpr int NCH = BZ ? 2 : 4;
  int ca[NCH], cm[NCH], nW[NCH], nE[NCH], nS[NCH], nN[NCH];
#pragma unroll
  for (int t = 0; t < NCH; ++t) {
    int a, bb;
    if (BZ) { a = t; bb = t; }                 // (0,0), (1,1)
    else { a = t & 1; bb = t >> 1; }
    const int i = 2 * I + a, j = 2 * J + bb;
    ca[t] = (a + bb) & 1;
    cm[t] = col_m(F, i, j);
    nW[t] = F.has_x ? col_m(F, wrapi(i - 1, F.nx), j) : 0;
    nE[t] = F.has_x ? col_m(F, wrapi(i + 1, F.nx), j) : 0;
    nS[t] = F.has_y ? col_m(F, i, wrapi(j - 1, F.ny)) : 0;
    nN[t] = F.has_y ? col_m(F, i, wrapi(j + 1, F.ny)) : 0;
  }
  const long long H = F.S;
  const R *__restrict__ tv = tab + TV * F.P;
  const R *__restrict__ tx = tab + TX * F.P;
  const R *__restrict__ ty = tab + TY * F.P;
  const R *__restrict__ tz = tab + TZ * F.P;
  const int nz = F.nz;

  R um[NCH], uc[NCH];
#pragma unroll
  for (int t = 0; t < NCH; ++t) {
    uc[t] = u[ca[t] * F.cs + cm[t]];
    um[t] = uc[t];
  }
  R *__restrict__ out = bc + (long long)cc * C.cs + mc;
  for (int k = 0; k < nz; ++k) {
    const long long o = (long long)k * H;
    R acc = R(0);
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
      const R *__restrict__ uo = u + (long long)(1 - ca[t]) * F.cs + o;
      const R *__restrict__ ow = u + (long long)ca[t] * F.cs;
      const R up = (k + 1 < nz) ? ow[o + H + cm[t]] : uc[t];
      const R uW = F.has_x ? uo[nW[t]] : R(0);
      const R uE = F.has_x ? uo[nE[t]] : R(0);
      const R uS = F.has_y ? uo[nS[t]] : R(0);
      const R uN = F.has_y ? uo[nN[t]] : R(0);
      const R bk = (R)b[(long long)ca[t] * F.cs + o + cm[t]];
      R tzlo, tzhi;
      if constexpr (C3) {
        const R *__restrict__ zc = tz3 + (long long)ca[t] * F.cs + cm[t];
        tzlo = zc[o];
        tzhi = k + 1 < nz ? zc[o + H] : R(0);
      } else {
        tzlo = tz[k];
        tzhi = tz[k + 1];
      }
      const R r = cell_residual<R>(bk, tv[k], tx[k], ty[k], tzlo, tzhi, uc[t], um[t], up,
                                   uW, uE, uS, uN, F.has_x, F.has_y);
      acc = t == 0 ? r : acc + r;
      um[t] = uc[t];
      uc[t] = up;
    }
    out[(long long)k * C.S] = acc;
  }
}

// -------------------------------------------------------------------------
// u += P uc (Sec. 6.2.1 "linear interpolation"): the fine cell centre lies a
// quarter coarse cell from its parent's centre, giving weights 9/16 (parent),
// 3/16 (the nearer x and y neighbours) and 1/16 (the diagonal one).
// MODE 1: piecewise constant.  RED_ONLY: colour-0 fine columns only.
// -------------------------------------------------------------------------
template <typename R, bool RED_ONLY, int MODE, int NSEG = kSeg>
__device__ __forceinline__ void prolong_body(Geo F, Geo C, const R *__restrict__ uc,
                                                    R *__restrict__ u,
                                                    const int *__restrict__ done, int lb, int nblocks) {
  if (is_done(done)) return;
  const int gid = lb * kSegCols + (threadIdx.x & 63);
  int c, m;
  if (RED_ONLY) {
    c = 0;
    m = gid;
    if (m >= F.ncol0) return;
  } else {
    if (gid >= 2 * F.H) return;
    c = gid & 1;
    m = gid >> 1;
    if (m >= (c ? F.ncol1 : F.ncol0)) return;
  }
  const int Ls = seg_len(F.nz, NSEG);
  const int k0 = min(wave_id() * Ls, F.nz), k1 = min(k0 + Ls, F.nz);
  int i, j;
  col_ij(F, c, m, i, j);
  const int I = i >> 1, J = j >> 1;
  const int I2 = wrapi(I + ((i & 1) ? 1 : -1), C.nx);
  const int J2 = wrapi(J + ((j & 1) ? 1 : -1), C.ny);
  const R *__restrict__ p11 = uc + (long long)((I + J) & 1) * C.cs + col_m(C, I, J);
  const R *__restrict__ p21 = uc + (long long)((I2 + J) & 1) * C.cs + col_m(C, I2, J);
  const R *__restrict__ p12 = uc + (long long)((I + J2) & 1) * C.cs + col_m(C, I, J2);
  const R *__restrict__ p22 = uc + (long long)((I2 + J2) & 1) * C.cs + col_m(C, I2, J2);
  R *__restrict__ own = u + (long long)c * F.cs + m;
  const long long HC = C.S, HF = F.S;
  auto interp = [&](R a, R b2, R c2, R d) -> R {
    if (MODE == 1) return a;
    R e = R(9.0 / 16.0) * a;
    e = e + R(3.0 / 16.0) * b2;
    e = e + R(3.0 / 16.0) * c2;
    e = e + R(1.0 / 16.0) * d;
    return e;
  };
  int k = k0;
  for (; k + kChunk <= k1; k += kChunk) {
    R o[kChunk], a[kChunk], b2[kChunk], c2[kChunk], d[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      const long long kc = (long long)(k + t) * HC;
      o[t] = own[(long long)(k + t) * HF];
      a[t] = p11[kc];
      if (MODE != 1) {
        b2[t] = p21[kc];
        c2[t] = p12[kc];
        d[t] = p22[kc];
      } else {
        b2[t] = c2[t] = d[t] = R(0);
      }
    }
#pragma unroll
    for (int t = 0; t < kChunk; ++t) own[(long long)(k + t) * HF] = o[t] + interp(a[t], b2[t], c2[t], d[t]);
  }
  for (; k < k1; ++k) {
    const long long kc = (long long)k * HC;
    const R e = MODE == 1 ? p11[kc] : interp(p11[kc], p21[kc], p12[kc], p22[kc]);
    own[(long long)k * HF] = own[(long long)k * HF] + e;
  }
}

// Colour-0 bilinear prolongation with the coarse values staged in LDS.  The
// column kernel's four coarse loads per level go through the texture units
// for every fine cell although each coarse value serves four fine cells; here
// a wavefront owns 32 m-columns by 2 rows of fine red cells (rows j0, j0+1
// share the coarse parent row J = j0/2) over one k-segment, and per level
// loads its own values and the coarse rows J-1, J, J+1 at coarse columns
// mx0-1 .. mx0+32 (102 values, two loads), then interpolates from LDS with
// the column kernel's weights and order (bitwise equal results).  Needs ny
// even and nx > 1; blocks past the last tile return at once.
// TO != R (the mixed-precision V-cycle's last prolongation): the corrected
// values go to out (of type TO) instead of back into u, as in prolong_out_body.
template <typename R, int NSEG, typename TO = R>
__device__ __forceinline__ void prolong_tile_body(Geo F, Geo C, const R *__restrict__ uc, R *__restrict__ u,
                                                  const int *__restrict__ done, int lb,
                                                  TO *__restrict__ out = nullptr) {
  __shared__ R cs[NSEG][3][36];
  const int tiles_x = (F.hx2 + kSTX - 1) / kSTX;
  if (is_done(done) || lb >= tiles_x * (F.ny / 2)) return;
  const int lane = threadIdx.x & 63;
  const int sg = wave_id();
  const int ty = lb / tiles_x, tx = lb - ty * tiles_x;
  const int mx0 = tx * kSTX, j0 = ty * 2;
  const int nxm = min(kSTX, F.hx2 - mx0);
  const int x = lane & 31, r = lane >> 5;
  const bool valid = x < nxm;
  const long long mo = (long long)(j0 + r) * F.hx2 + mx0 + (valid ? x : nxm - 1);
  const int J = j0 >> 1;
  // staged coarse values: v = lane (first load) and 64 + lane (second); row v/34, column v%34
  auto coarse_off = [&](int v, bool &need) -> long long {
    const int row = v / 34, q = v - row * 34;
    need = v < 102 && q <= nxm + 1;
    const int I = wrapi(mx0 - 1 + (need ? q : 1), C.nx);
    const int Jr = wrapi(J - 1 + (need ? row : 1), C.ny);
    return (long long)((I + Jr) & 1) * C.cs + col_m(C, I, Jr);
  };
  bool need0, need1;
  const long long co0 = coarse_off(lane, need0), co1 = coarse_off(64 + lane, need1);
  const int r0 = lane / 34, q0 = lane - r0 * 34, r1 = (64 + lane) / 34, q1 = (64 + lane) - r1 * 34;
  const long long HC = C.S, HF = F.S;
  const int nz = F.nz, Ls = seg_len(nz, NSEG);
  const int k0 = min(sg * Ls, nz), k1 = min(k0 + Ls, nz);
  R(*slot)[36] = cs[sg];
  // the four coarse neighbours of this lane's fine cell in the slot
  const int ia = x + 1, ib = r ? x + 2 : x, rc = r ? 2 : 0;
  R *__restrict__ own = u + mo;
  for (int k = k0; k < k1; k += kChunk) {
    R o[kChunk], v0[kChunk], v1[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      const int kk = min(k + t, k1 - 1);
      o[t] = __builtin_nontemporal_load(&own[(long long)kk * HF]);
      v0[t] = uc[(long long)kk * HC + co0];
      v1[t] = need1 ? uc[(long long)kk * HC + co1] : R(0);
    }
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      if (k + t < k1) {
        if (need0) slot[r0][q0] = v0[t];
        if (need1) slot[r1][q1] = v1[t];
        __asm__ volatile("" ::: "memory");
        const R a = slot[1][ia], b2 = slot[1][ib], c2 = slot[rc][ia], d = slot[rc][ib];
        __asm__ volatile("" ::: "memory");
        R e = R(9.0 / 16.0) * a;
        e = e + R(3.0 / 16.0) * b2;
        e = e + R(3.0 / 16.0) * c2;
        e = e + R(1.0 / 16.0) * d;
        if (valid) {
          if constexpr (std::is_same<R, TO>::value) own[(long long)(k + t) * HF] = o[t] + e;
          else out[mo + (long long)(k + t) * HF] = (TO)o[t] + (TO)e;
        }
      }
    }
  }
}

template <typename R, int NSEG>
__global__ __launch_bounds__(NSEG * 64) void k_prolong_tile(Geo F, Geo C, const R *__restrict__ uc,
                                                            R *__restrict__ u, const int *__restrict__ done) {
  prolong_tile_body<R, NSEG>(F, C, uc, u, done, logical_block());
}

// The mixed-precision V-cycle's last prolongation on the tile: out = base +
// P e_c on colour 0 (FP32 base and correction, FP64 out), bitwise equal to
// k_prolong_out.
template <typename R, typename TO, int NSEG>
__global__ __launch_bounds__(NSEG * 64) void k_prolong_out_tile(Geo F, Geo C, const R *__restrict__ uc,
                                                                const R *__restrict__ base, TO *__restrict__ out,
                                                                const int *__restrict__ done) {
  prolong_tile_body<R, NSEG, TO>(F, C, uc, const_cast<R *>(base), done, logical_block(), out);
}

template <typename R, bool RED_ONLY, int MODE, int NSEG = kSeg>
__global__ __launch_bounds__(NSEG * 64) void k_prolong(Geo F, Geo C, const R *__restrict__ uc,
                                                       R *__restrict__ u,
                                                       const int *__restrict__ done) {
  prolong_body<R, RED_ONLY, MODE, NSEG>(F, C, uc, u, done, logical_block(), gridDim.x);
}

// Colour-0 prolongation from an FP32 hierarchy into the FP64 output of the
// finest level: out = base + P uc on colour-0 columns (base: the FP32
// pre-smoothed iterate).  Bilinear weights as in k_prolong.
template <typename R, typename TO, int MODE>
__device__ __forceinline__ void prolong_out_body(Geo F, Geo C, const R *__restrict__ uc,
                                                        const R *__restrict__ base,
                                                        TO *__restrict__ out,
                                                        const int *__restrict__ done, int lb, int nblocks) {
  if (is_done(done)) return;
  const int m = lb * kSegCols + (threadIdx.x & 63);
  if (m >= F.ncol0) return;
  const int Ls = seg_len(F.nz);
  const int k0 = min(wave_id() * Ls, F.nz), k1 = min(k0 + Ls, F.nz);
  int i, j;
  col_ij(F, 0, m, i, j);
  const int I = i >> 1, J = j >> 1;
  const int I2 = wrapi(I + ((i & 1) ? 1 : -1), C.nx);
  const int J2 = wrapi(J + ((j & 1) ? 1 : -1), C.ny);
  const R *__restrict__ p11 = uc + (long long)((I + J) & 1) * C.cs + col_m(C, I, J);
  const R *__restrict__ p21 = uc + (long long)((I2 + J) & 1) * C.cs + col_m(C, I2, J);
  const R *__restrict__ p12 = uc + (long long)((I + J2) & 1) * C.cs + col_m(C, I, J2);
  const R *__restrict__ p22 = uc + (long long)((I2 + J2) & 1) * C.cs + col_m(C, I2, J2);
  const R *__restrict__ bs = base + m;
  TO *__restrict__ ow = out + m;
  const long long HC = C.S, HF = F.S;
#pragma unroll 4
  for (int k = k0; k < k1; ++k) {
    const long long kc = (long long)k * HC;
    R e;
    if (MODE == 1) {
      e = p11[kc];
    } else {
      e = R(9.0 / 16.0) * p11[kc];
      e = e + R(3.0 / 16.0) * p21[kc];
      e = e + R(3.0 / 16.0) * p12[kc];
      e = e + R(1.0 / 16.0) * p22[kc];
    }
    ow[(long long)k * HF] = (TO)bs[(long long)k * HF] + (TO)e;
  }
}

template <typename R, typename TO, int MODE>
__global__ __launch_bounds__(kBlock) void k_prolong_out(Geo F, Geo C, const R *__restrict__ uc,
                                                        const R *__restrict__ base,
                                                        TO *__restrict__ out,
                                                        const int *__restrict__ done) {
  prolong_out_body<R, TO, MODE>(F, C, uc, base, out, done, logical_block(), gridDim.x);
}

// -------------------------------------------------------------------------
// y = A x (eq. ModelEquation integrated over the cell, difference form), one
// lane per column of either colour; DOT: also partial sums of <x, y>.
// -------------------------------------------------------------------------
template <typename R, bool DOT, bool HXY, int NSEG, bool C3 = false>
__global__ __launch_bounds__(kBlock) void k_apply(Geo L, const R *__restrict__ tab,
                                                  const R *__restrict__ x, R *__restrict__ y,
                                                  double *__restrict__ partial,
                                                  const int *__restrict__ done,
                                                  const R *__restrict__ tz3 = nullptr) {
  __shared__ double sh[4];
  if (is_done(done)) return;
  // 64 column slots (both colours) per block, one k-segment per wavefront
  // lanes alternate colours: the red and black columns of one stretch of a
  // row (each other's neighbours) are handled by the same wavefront
  constexpr int CH = 4 / NSEG;  // 64-slot chunks per block
  const int w = wave_id();
  const int sg = w / CH;
  const int slot = (logical_block() * CH + (w % CH)) * kSegCols + (threadIdx.x & 63);
  const int c = slot & 1;
  const int m = slot >> 1;
  const bool valid = slot < 2 * L.H && m < (c ? L.ncol1 : L.ncol0);
  const int Ls = seg_len(L.nz, NSEG);
  const int k0 = min(sg * Ls, L.nz), k1 = min(k0 + Ls, L.nz);
  double dot = 0.0;
  if (valid && k1 > k0) {
    int i, j;
    col_ij(L, c, m, i, j);
    const Nbr nb = neighbours(L, i, j);
    const bool hx = HXY || L.has_x, hy = HXY || L.has_y;
    const long long H = L.S;
    const R *__restrict__ xo = x + (long long)(1 - c) * L.cs;
    const R *__restrict__ xw = xo + nb.w;
    const R *__restrict__ xe = xo + nb.e;
    const R *__restrict__ xs_ = xo + nb.s;
    const R *__restrict__ xn = xo + nb.n;
    const R *__restrict__ xs = x + (long long)c * L.cs + m;
    R *__restrict__ ys = y + (long long)c * L.cs + m;
    const R *__restrict__ tv = tab + TV * L.P;
    const R *__restrict__ tx = tab + TX * L.P;
    const R *__restrict__ ty = tab + TY * L.P;
    const R *__restrict__ tz = tab + TZ * L.P;
    const int nz = L.nz;
    const R *__restrict__ zc = C3 ? tz3 + (long long)c * L.cs + m : nullptr;  // this column's faces
    auto cell = [&](int k, R xc, R xm, R xp, R w, R e, R so, R no) -> R {
      R acc = tv[k] * xc;
      if (hx) {
        acc = acc + tx[k] * (xc - w);
        acc = acc + tx[k] * (xc - e);
      }
      if (hy) {
        acc = acc + ty[k] * (xc - so);
        acc = acc + ty[k] * (xc - no);
      }
      if constexpr (C3) {
        acc = acc + zc[(long long)k * H] * (xc - xm);
        acc = acc + (k + 1 < nz ? zc[(long long)(k + 1) * H] : R(0)) * (xc - xp);
      } else {
        acc = acc + tz[k] * (xc - xm);
        acc = acc + tz[k + 1] * (xc - xp);
      }
      return acc;
    };
    R xc = xs[(long long)k0 * H];
    R xm = k0 > 0 ? xs[(long long)(k0 - 1) * H] : xc;
    int k = k0;
    for (; k + kChunk <= k1; k += kChunk) {
      R xp[kChunk], w[kChunk], e[kChunk], so[kChunk], no[kChunk];
#pragma unroll
      for (int t = 0; t < kChunk; ++t) {
        const long long o = (long long)(k + t) * H;
        const int kp = min(k + t + 1, nz - 1);
        xp[t] = xs[(long long)kp * H];
        w[t] = hx ? xw[o] : R(0);
        e[t] = hx ? xe[o] : R(0);
        so[t] = hy ? xs_[o] : R(0);
        no[t] = hy ? xn[o] : R(0);
      }
#pragma unroll
      for (int t = 0; t < kChunk; ++t) {
        const R acc = cell(k + t, xc, xm, xp[t], w[t], e[t], so[t], no[t]);
        ys[(long long)(k + t) * H] = acc;
        if (DOT) dot += (double)xc * (double)acc;
        xm = xc;
        xc = xp[t];
      }
    }
    for (; k < k1; ++k) {
      const long long o = (long long)k * H;
      const R xpv = xs[(long long)min(k + 1, nz - 1) * H];
      const R acc = cell(k, xc, xm, xpv, hx ? xw[o] : R(0), hx ? xe[o] : R(0), hy ? xs_[o] : R(0),
                         hy ? xn[o] : R(0));
      ys[o] = acc;
      if (DOT) dot += (double)xc * (double)acc;
      xm = xc;
      xc = xpv;
    }
  }
  if (DOT) {
    const double s = block_sum(dot, sh);
    if (threadIdx.x == 0) partial[logical_block()] = s;
  }
}

// -------------------------------------------------------------------------
// One CG step's vector work around the operator (Appendix B, Alg. PCG):
//   p_new = z + beta p_old          (search direction; p_new = z when first)
//   q     = A p_new, partial sums of <p_new, q>
//   defer_u = 1: u += alpha p_old   (the previous step's solution update,
//                                    deferred to ride on the p_old read)
//   defer_u = 2: u = (u + alpha_prev p_old2) + alpha p_old
//                                   (the updates of the two previous steps,
//                                    in their order: every other step reads
//                                    and writes u once for two updates)
// alpha / alpha_prev: the step lengths of p_old / p_old2.  p_old2, p_old and
// p_new are different buffers, so neighbour values of p_new are formed from
// z and p_old exactly as their owning lanes form them.
// -------------------------------------------------------------------------
// C3: the vertical faces of each column from the split-layout field tz3
// (T_{k-1/2}) instead of the table.
template <typename Z, int NSEG, bool C3 = false>
__device__ __forceinline__ void apply_dir_body(Geo L, const double *__restrict__ tab,
                                                      const Z *__restrict__ z,
                                                      const double *__restrict__ pold,
                                                      const double *__restrict__ pold2,
                                                      double *__restrict__ pnew,
                                                      double *__restrict__ q,
                                                      double *__restrict__ u,
                                                      const PcgState *__restrict__ st, int first,
                                                      int defer_u, double *__restrict__ partial, int lb, int nblocks,
                                                      const double *__restrict__ tz3 = nullptr) {
  constexpr int U = 4;
  constexpr int CH = 4 / NSEG;
  __shared__ double sh[4];
  if (st->done) return;
  const double beta = first ? 0.0 : st->beta;
  const double alpha = st->alpha, alpha2 = st->alpha_prev;
  const int w = wave_id();
  const int sg = w / CH;
  const int slot = (lb * CH + (w % CH)) * kSegCols + (threadIdx.x & 63);
  const int c = slot & 1;
  const int m = slot >> 1;
  const bool valid = slot < 2 * L.H && m < (c ? L.ncol1 : L.ncol0);
  const int Ls = seg_len(L.nz, NSEG);
  const int k0 = min(sg * Ls, L.nz), k1 = min(k0 + Ls, L.nz);
  double dot = 0.0;
  if (valid && k1 > k0) {
    int i, j;
    col_ij(L, c, m, i, j);
    const Nbr nb = neighbours(L, i, j);
    const bool hx = L.has_x, hy = L.has_y;
    const long long H = L.S;
    const long long oo = (long long)(1 - c) * L.cs, os = (long long)c * L.cs + m;
    const double *__restrict__ tv = tab + TV * L.P;
    const double *__restrict__ tx = tab + TX * L.P;
    const double *__restrict__ ty = tab + TY * L.P;
    const double *__restrict__ tz = tab + TZ * L.P;
    const int nz = L.nz;
    // direction value at (column offset, level): z + beta p_old
    auto dir = [&](long long idx) -> double {
      return first ? (double)z[idx] : (double)z[idx] + beta * pold[idx];
    };
    // faces below and above level k of this column
    auto tlo = [&](int k) -> double { if constexpr (C3) return tz3[os + (long long)k * H]; else return tz[k]; };
    auto thi = [&](int k) -> double {
      if constexpr (C3) return k + 1 < nz ? tz3[os + (long long)(k + 1) * H] : 0.0;
      else return tz[k + 1];
    };
    auto cell = [&](int k, double zlo, double zhi, double pc, double pm, double pp, double pw, double pe,
                    double ps, double pn) -> double {
      double acc = tv[k] * pc;
      if (hx) {
        acc = acc + tx[k] * (pc - pw);
        acc = acc + tx[k] * (pc - pe);
      }
      if (hy) {
        acc = acc + ty[k] * (pc - ps);
        acc = acc + ty[k] * (pc - pn);
      }
      acc = acc + zlo * (pc - pm);
      acc = acc + zhi * (pc - pp);
      return acc;
    };
    double pc = dir(os + (long long)k0 * H);
    double pm = k0 > 0 ? dir(os + (long long)(k0 - 1) * H) : pc;
    int k = k0;
    for (; k + U <= k1; k += U) {
      double pp[U], pw[U], pe[U], ps[U], pn[U], uu[U], po[U], p2[U], zl[U], zh[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const long long o = (long long)(k + t) * H;
        zl[t] = tlo(k + t);
        zh[t] = thi(k + t);
        pp[t] = dir(os + (long long)min(k + t + 1, nz - 1) * H);
        pw[t] = hx ? dir(oo + nb.w + o) : 0.0;
        pe[t] = hx ? dir(oo + nb.e + o) : 0.0;
        ps[t] = hy ? dir(oo + nb.s + o) : 0.0;
        pn[t] = hy ? dir(oo + nb.n + o) : 0.0;
        uu[t] = defer_u ? u[os + o] : 0.0;
        po[t] = defer_u ? pold[os + o] : 0.0;
        p2[t] = defer_u == 2 ? pold2[os + o] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const long long o = (long long)(k + t) * H;
        const double acc = cell(k + t, zl[t], zh[t], pc, pm, pp[t], pw[t], pe[t], ps[t], pn[t]);
        q[os + o] = acc;
        pnew[os + o] = pc;
        if (defer_u) {
          double nu = uu[t];
          if (defer_u == 2) nu = nu + alpha2 * p2[t];
          u[os + o] = nu + alpha * po[t];
        }
        dot += pc * acc;
        pm = pc;
        pc = pp[t];
      }
    }
    for (; k < k1; ++k) {
      const long long o = (long long)k * H;
      const double pp = dir(os + (long long)min(k + 1, nz - 1) * H);
      const double acc = cell(k, tlo(k), thi(k), pc, pm, pp, hx ? dir(oo + nb.w + o) : 0.0,
                              hx ? dir(oo + nb.e + o) : 0.0, hy ? dir(oo + nb.s + o) : 0.0,
                              hy ? dir(oo + nb.n + o) : 0.0);
      q[os + o] = acc;
      pnew[os + o] = pc;
      if (defer_u) {
        double nu = u[os + o];
        if (defer_u == 2) nu = nu + alpha2 * pold2[os + o];
        u[os + o] = nu + alpha * pold[os + o];
      }
      dot += pc * acc;
      pm = pc;
      pc = pp;
    }
  }
  const double s = block_sum(dot, sh);
  if (threadIdx.x == 0) partial[lb] = s;
}

template <typename Z, int NSEG, bool C3 = false>
__global__ __launch_bounds__(kBlock) void k_apply_dir(Geo L, const double *__restrict__ tab,
                                                      const Z *__restrict__ z,
                                                      const double *__restrict__ pold,
                                                      const double *__restrict__ pold2,
                                                      double *__restrict__ pnew,
                                                      double *__restrict__ q,
                                                      double *__restrict__ u,
                                                      const PcgState *__restrict__ st, int first,
                                                      int defer_u, double *__restrict__ partial,
                                                      const double *__restrict__ tz3 = nullptr) {
  apply_dir_body<Z, NSEG, C3>(L, tab, z, pold, pold2, pnew, q, u, st, first, defer_u, partial, logical_block(),
                              gridDim.x, tz3);
}

// r <- r - alpha q, partial sums of ||r||^2
__device__ __forceinline__ void update_r_body(double2 *__restrict__ r,
                                                     const double2 *__restrict__ q, long long n2,
                                                     const PcgState *__restrict__ st,
                                                     double *__restrict__ partial, int lb, int nblocks) {
  __shared__ double sh[4];
  if (st->done) return;
  const double alpha = st->alpha;
  const long long t = (long long)lb * kBlock + threadIdx.x;
  const long long stride = (long long)nblocks * kBlock;
  double rr = 0.0;
  for (long long e = t; e < n2; e += stride) {
    const double2 qv = ld_nt(&q[e]);
    double2 rv = ld_nt(&r[e]);
    rv.x = rv.x - alpha * qv.x;
    rv.y = rv.y - alpha * qv.y;
    st_nt(&r[e], rv);
    rr += rv.x * rv.x + rv.y * rv.y;
  }
  const double s = block_sum(rr, sh);
  if (threadIdx.x == 0) partial[lb] = s;
}

__global__ __launch_bounds__(kBlock) void k_update_r(double2 *__restrict__ r,
                                                     const double2 *__restrict__ q, long long n2,
                                                     const PcgState *__restrict__ st,
                                                     double *__restrict__ partial) {
  update_r_body(r, q, n2, st, partial, logical_block(), gridDim.x);
}

// A fixed pseudo-random field in [-1, 1): element e is a 64-bit mix of e
// (the input of schedule timing; nothing numerical depends on its values).
__global__ __launch_bounds__(kBlock) void k_fill_hash(double *__restrict__ f, long long n) {
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += stride) {
    unsigned long long x = (unsigned long long)e * 0x9E3779B97F4A7C15ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    f[e] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_fill(R *__restrict__ p, long long n, R v) {
  const long long t = (long long)logical_block() * kBlock + threadIdx.x;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = t; e < n; e += stride) p[e] = v;
}

// plane-major -> colour-split, optionally scaled by the cell volume V_k
template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_nat2split(Geo L, const S *__restrict__ src,
                                                      D *__restrict__ dst,
                                                      const double *__restrict__ vol) {
  const int gid = logical_block() * kBlock + threadIdx.x;
  if (gid >= 2 * L.H) return;
  const int c = gid >= L.H ? 1 : 0;
  const int m = gid - c * L.H;
  if (m >= (c ? L.ncol1 : L.ncol0)) return;
  int i, j;
  col_ij(L, c, m, i, j);
  const long long plane = (long long)L.nx * L.ny;
  for (int k = 0; k < L.nz; ++k) {
    double v = (double)src[k * plane + (long long)j * L.nx + i];
    if (vol) v = vol[k] * v;
    dst[(long long)c * L.cs + (long long)k * L.S + m] = (D)v;
  }
}

template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_split2nat(Geo L, const S *__restrict__ src,
                                                      D *__restrict__ dst) {
  const int gid = logical_block() * kBlock + threadIdx.x;
  if (gid >= 2 * L.H) return;
  const int c = gid >= L.H ? 1 : 0;
  const int m = gid - c * L.H;
  if (m >= (c ? L.ncol1 : L.ncol0)) return;
  int i, j;
  col_ij(L, c, m, i, j);
  const long long plane = (long long)L.nx * L.ny;
  for (int k = 0; k < L.nz; ++k)
    dst[k * plane + (long long)j * L.nx + i] = (D)src[(long long)c * L.cs + (long long)k * L.S + m];
}

// FP64 residual -> FP32 right-hand side of the preconditioner
__global__ __launch_bounds__(kBlock) void k_cast_f64_f32(const double2 *__restrict__ src,
                                                         float2 *__restrict__ dst, long long n2,
                                                         const int *__restrict__ done) {
  if (is_done(done)) return;
  const long long t = (long long)logical_block() * kBlock + threadIdx.x;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = t; e < n2; e += stride) {
    const double2 v = src[e];
    dst[e] = make_float2((float)v.x, (float)v.y);
  }
}

// -------------------------------------------------------------------------
// The same fused operator step on horizontal tiles staged in LDS.  A block
// owns a tile of kTX x kTY columns per colour (64 x 16 plane-major columns)
// over one k-segment and walks it level by level.  The direction values
// p = z + beta p_old of a level, for the tile and its one-cell horizontal
// halo, are formed once and put in LDS; the horizontal neighbours are read
// from there and the vertical ones from registers, so each z and p_old value
// is fetched by one block (halo values by two) instead of by up to five
// wavefronts at different times.  LDS holds the tile per colour in the split
// order (row-major, m-contiguous), so lanes of a wavefront touch consecutive
// LDS words and consecutive memory.  Three LDS buffers rotate: one barrier
// per level separates the writes of level k+1 from the reads of level k.
// Requires nx and ny even (both horizontal directions present).  Blocks
// (tiles x segments) past the end write zero partial sums.
// -------------------------------------------------------------------------
constexpr int kTX = 32;  // tile width per colour (m-columns)
constexpr int kTY = 16;  // tile rows
constexpr int kTW = kTX + 2, kTH = kTY + 2;

__host__ __device__ inline int tile_count(int hx2, int ny) {
  return ((hx2 + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY);
}

// C3: the vertical faces of each own cell from the split-layout field tz3
// (T_{k-1/2}), loaded with the level they belong to.
template <typename Z, bool C3 = false>
__device__ __forceinline__ void apply_dir_tile_body(Geo L, int nseg, const double *__restrict__ tab,
                                                    const Z *__restrict__ z,
                                                    const double *__restrict__ pold,
                                                    const double *__restrict__ pold2,
                                                    double *__restrict__ pnew, double *__restrict__ q,
                                                    double *__restrict__ u,
                                                    const PcgState *__restrict__ st, int first,
                                                    int defer_u, double *__restrict__ partial, int lb,
                                                    const double *__restrict__ tz3 = nullptr) {
  __shared__ double sp[3][2][kTH][kTW];
  __shared__ double sh[4];
  if (st->done) return;
  const double beta = first ? 0.0 : st->beta;
  const double alpha = st->alpha, alpha2 = st->alpha_prev;
  const int tiles_x = (L.hx2 + kTX - 1) / kTX;
  const int per_seg = tile_count(L.hx2, L.ny);
  const int sg = lb / per_seg, tt = lb - sg * per_seg;
  const int ty = tt / tiles_x, tx = tt - ty * tiles_x;
  const int Ls = seg_len(L.nz, nseg);
  const int k0 = min(sg * Ls, L.nz), k1 = min(k0 + Ls, L.nz);
  double dot = 0.0;
  if (k1 > k0) {
    const int t = threadIdx.x;
    const int mx0 = tx * kTX, j0 = ty * kTY;
    const int nxm = min(kTX, L.hx2 - mx0);  // valid m-columns of the tile
    const int nyr = min(kTY, L.ny - j0);    // valid rows of the tile
    const int x = t & 31, r0 = t >> 5;      // own cells: rows r0 and r0 + 8, both colours
    const long long S = L.S, cs = L.cs;
    long long off[4];
    bool ok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = e & 1, rr = r0 + 8 * (e >> 1);
      ok[e] = x < nxm && rr < nyr;
      off[e] = (long long)c * cs + (long long)(j0 + rr) * L.hx2 + mx0 + x;
    }
    // one halo cell per thread for threads 0..159: rows below / above the
    // tile (both colours), then the cells left / right of each row
    bool hok = false;
    long long hoff = 0;
    int hc = 0, hr = 0, hx = 0;
    if (t < 128) {
      const int side = t >> 6, c = (t >> 5) & 1, xx = t & 31;
      const int j = side ? wrapi(j0 + nyr, L.ny) : wrapi(j0 - 1, L.ny);
      hok = xx < nxm;
      hoff = (long long)c * cs + (long long)j * L.hx2 + mx0 + xx;
      hc = c;
      hr = side ? nyr + 1 : 0;
      hx = xx + 1;
    } else if (t < 160) {
      const int side = (t - 128) >> 4, rr = (t - 128) & 15;
      const int j = j0 + rr;
      const int i = side ? wrapi(2 * (mx0 + nxm), L.nx) : wrapi(2 * mx0 - 1, L.nx);
      const int c = (i + j) & 1;
      hok = rr < nyr;
      hoff = (long long)c * cs + (long long)j * L.hx2 + (i >> 1);
      hc = c;
      hr = rr + 1;
      hx = side ? nxm + 1 : 0;
    }
    auto dirv = [&](long long idx) -> double {
      return first ? (double)z[idx] : (double)z[idx] + beta * pold[idx];
    };
    // level k: own direction values into pv (and LDS buffer b when b >= 0);
    // with write set, also p_new and the deferred solution update
    auto level = [&](int k, int b, bool write, double *pv) {
      const long long o = (long long)k * S;
      double zv[4], po[4], uu[4], p2[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        zv[e] = ok[e] ? (double)z[off[e] + o] : 0.0;
        po[e] = (ok[e] && !first) ? pold[off[e] + o] : 0.0;
        uu[e] = (ok[e] && write && defer_u) ? __builtin_nontemporal_load(&u[off[e] + o]) : 0.0;
        p2[e] = (ok[e] && write && defer_u == 2) ? __builtin_nontemporal_load(&pold2[off[e] + o]) : 0.0;
      }
      double hv = 0.0;
      if (b >= 0 && hok) hv = dirv(hoff + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double pvv = first ? zv[e] : zv[e] + beta * po[e];
        pv[e] = pvv;
        // only valid cells: in a partial tile the slots past the last valid
        // row / m-column hold the halo
        if (b >= 0 && ok[e]) sp[b][e & 1][r0 + 8 * (e >> 1) + 1][x + 1] = pvv;
        if (ok[e] && write) {
          __builtin_nontemporal_store(pvv, &pnew[off[e] + o]);
          if (defer_u) {
            // the older update first: the same two steps as one per iteration
            double nu = uu[e];
            if (defer_u == 2) nu = nu + alpha2 * p2[e];
            nu = nu + alpha * po[e];
            __builtin_nontemporal_store(nu, &u[off[e] + o]);
          }
        }
      }
      if (b >= 0 && hok) sp[b][hc][hr][hx] = hv;
    };
    const double *__restrict__ tv = tab + TV * L.P;
    const double *__restrict__ txv = tab + TX * L.P;
    const double *__restrict__ tyv = tab + TY * L.P;
    const double *__restrict__ tz = tab + TZ * L.P;
    // C3: faces below the own cells of level kk (the face above level kk - 1)
    double fzc[4] = {0.0, 0.0, 0.0, 0.0}, fzn[4] = {0.0, 0.0, 0.0, 0.0};
    auto faces = [&](int kk, double *fz) {
      if constexpr (C3) {
#pragma unroll
        for (int e = 0; e < 4; ++e) fz[e] = ok[e] ? tz3[off[e] + (long long)kk * S] : 0.0;
      }
    };
    double pm[4], pc[4], pn[4];
    level(k0, k0 % 3, true, pc);
    faces(k0, fzc);
    if (k0 > 0) level(k0 - 1, -1, false, pm);
    else {
#pragma unroll
      for (int e = 0; e < 4; ++e) pm[e] = pc[e];
    }
    for (int k = k0; k < k1; ++k) {
      if (k + 1 < k1) {
        level(k + 1, (k + 1) % 3, true, pn);
        faces(k + 1, fzn);
      } else if (k + 1 < L.nz) {
        level(k + 1, -1, false, pn);
        faces(k + 1, fzn);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          pn[e] = pc[e];
          fzn[e] = 0.0;
        }
      }
      __syncthreads();
      const int b = k % 3;
      const long long o = (long long)k * S;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (ok[e]) {
          const int c = e & 1, rr = r0 + 8 * (e >> 1);
          const int par = (j0 + rr + c) & 1;  // 1: the cell sits at an odd i
          const double(*oth)[kTW] = sp[b][1 - c];
          const double pw = oth[rr + 1][x + par];
          const double pe = oth[rr + 1][x + 1 + par];
          const double ps = oth[rr][x + 1];
          const double pnn = oth[rr + 2][x + 1];
          const double pcv = pc[e];
          double acc = tv[k] * pcv;
          acc = acc + txv[k] * (pcv - pw);
          acc = acc + txv[k] * (pcv - pe);
          acc = acc + tyv[k] * (pcv - ps);
          acc = acc + tyv[k] * (pcv - pnn);
          if constexpr (C3) {
            acc = acc + fzc[e] * (pcv - pm[e]);
            acc = acc + fzn[e] * (pcv - pn[e]);
          } else {
            acc = acc + tz[k] * (pcv - pm[e]);
            acc = acc + tz[k + 1] * (pcv - pn[e]);
          }
          __builtin_nontemporal_store(acc, &q[off[e] + o]);
          dot += pcv * acc;
        }
        pm[e] = pc[e];
        pc[e] = pn[e];
        fzc[e] = fzn[e];
      }
    }
  }
  const double s = block_sum(dot, sh);
  if (threadIdx.x == 0) partial[lb] = s;
}

template <typename Z, bool C3 = false>
__global__ __launch_bounds__(kBlock) void k_apply_dir_tile(Geo L, int nseg, const double *__restrict__ tab,
                                                           const Z *__restrict__ z,
                                                           const double *__restrict__ pold,
                                                           const double *__restrict__ pold2,
                                                           double *__restrict__ pnew, double *__restrict__ q,
                                                           double *__restrict__ u,
                                                           const PcgState *__restrict__ st, int first,
                                                           int defer_u, double *__restrict__ partial,
                                                           const double *__restrict__ tz3 = nullptr) {
  apply_dir_tile_body<Z, C3>(L, nseg, tab, z, pold, pold2, pnew, q, u, st, first, defer_u, partial, logical_block(),
                             tz3);
}

// -------------------------------------------------------------------------
// Start and end of a solve, one pass each (Appendix B, Alg. PCG: initial
// residual, final solution).  Both evaluate the operator exactly as the
// split-layout operator kernel does (same terms in the same order), with
// f and u in plane-major order [k][j][i] at the library boundary.
// -------------------------------------------------------------------------

// Operator row of one cell (eq. (FV) with the harmonic vertical faces):
// V_k u_c + Tx_k (2 u_c - u_W - u_E) + Ty_k (2 u_c - u_S - u_N)
//         + T_{k-1/2} (u_c - u_{k-1}) + T_{k+1/2} (u_c - u_{k+1}).
__device__ __forceinline__ double op_row(const double *__restrict__ tab, int P, int k, bool hx, bool hy,
                                         double uc, double um, double up, double uw, double ue,
                                         double us, double un) {
  double acc = tab[TV * P + k] * uc;
  if (hx) {
    acc = acc + tab[TX * P + k] * (uc - uw);
    acc = acc + tab[TX * P + k] * (uc - ue);
  }
  if (hy) {
    acc = acc + tab[TY * P + k] * (uc - us);
    acc = acc + tab[TY * P + k] * (uc - un);
  }
  acc = acc + tab[TZ * P + k] * (uc - um);
  acc = acc + tab[TZ * P + k + 1] * (uc - up);
  return acc;
}

// The same row with the two vertical faces given (per-column coefficients).
__device__ __forceinline__ double op_row_v(const double *__restrict__ tab, int P, int k, bool hx, bool hy,
                                           double tzlo, double tzhi, double uc, double um, double up,
                                           double uw, double ue, double us, double un) {
  double acc = tab[TV * P + k] * uc;
  if (hx) {
    acc = acc + tab[TX * P + k] * (uc - uw);
    acc = acc + tab[TX * P + k] * (uc - ue);
  }
  if (hy) {
    acc = acc + tab[TY * P + k] * (uc - us);
    acc = acc + tab[TY * P + k] * (uc - un);
  }
  acc = acc + tzlo * (uc - um);
  acc = acc + tzhi * (uc - up);
  return acc;
}

// us = u0 and r = V f - A u0 in the split layout, from plane-major f and u0;
// partial[2 lb] = sum (V f)^2, partial[2 lb + 1] = sum r^2 over the block.
// One block = 64 plane-major columns (lanes are consecutive i: every
// plane-major access is coalesced, and each colour receives 32 consecutive
// split entries per wavefront), one k-segment of four per wavefront.
// Blocks past the last column write zero partial sums.
// C3: the vertical faces of each column from the split-layout field tz3.
template <bool C3 = false>
__device__ __forceinline__ void begin_body(Geo L, const double *__restrict__ tab,
                                           const double *__restrict__ vol,
                                           const double *__restrict__ f,
                                           const double *__restrict__ u0, double *__restrict__ us,
                                           double *__restrict__ r, double *__restrict__ partial,
                                           int lb, const double *__restrict__ tz3 = nullptr) {
  constexpr int NSEG = 4, U = 4;
  __shared__ double sh[4];
  const int sg = wave_id();
  const long long plane = (long long)L.nx * L.ny;
  const long long col = (long long)lb * kSegCols + (threadIdx.x & 63);
  const int Ls = seg_len(L.nz, NSEG);
  const int k0 = min(sg * Ls, L.nz), k1 = min(k0 + Ls, L.nz);
  double bb = 0.0, rr = 0.0;
  if (col < plane && k1 > k0) {
    const int j = (int)(col / L.nx), i = (int)(col - (long long)j * L.nx);
    const int c = (i + j) & 1;
    const long long m = col_m(L, i, j);
    const bool hx = L.has_x, hy = L.has_y;
    const long long oc = col;
    const long long ow = hx ? (long long)j * L.nx + wrapi(i - 1, L.nx) : oc;
    const long long oe = hx ? (long long)j * L.nx + wrapi(i + 1, L.nx) : oc;
    const long long osn = hy ? (long long)wrapi(j - 1, L.ny) * L.nx + i : oc;
    const long long onn = hy ? (long long)wrapi(j + 1, L.ny) * L.nx + i : oc;
    double *__restrict__ usc = us + (long long)c * L.cs + m;
    double *__restrict__ rc = r + (long long)c * L.cs + m;
    const long long S = L.S;
    const int nz = L.nz, P = L.P;
    double uc = u0[(long long)k0 * plane + oc];
    double um = k0 > 0 ? u0[(long long)(k0 - 1) * plane + oc] : uc;
    int k = k0;
    for (; k < k1; k += U) {
      double up[U], uw[U], ue[U], usv[U], un[U], fv[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const int kk = min(k + t, k1 - 1);
        const long long o = (long long)kk * plane;
        up[t] = u0[(long long)min(kk + 1, nz - 1) * plane + oc];
        uw[t] = hx ? u0[o + ow] : 0.0;
        ue[t] = hx ? u0[o + oe] : 0.0;
        usv[t] = hy ? u0[o + osn] : 0.0;
        un[t] = hy ? u0[o + onn] : 0.0;
        fv[t] = f[o + oc];
      }
#pragma unroll
      for (int t = 0; t < U; ++t) {
        if (k + t < k1) {
          const int kk = k + t;
          double acc;
          if constexpr (C3) {
            const double *__restrict__ zc = tz3 + (long long)c * L.cs + m;
            acc = op_row_v(tab, P, kk, hx, hy, zc[(long long)kk * S], kk + 1 < nz ? zc[(long long)(kk + 1) * S] : 0.0,
                           uc, um, up[t], uw[t], ue[t], usv[t], un[t]);
          } else {
            acc = op_row(tab, P, kk, hx, hy, uc, um, up[t], uw[t], ue[t], usv[t], un[t]);
          }
          const double b = vol[kk] * fv[t];
          const double res = b - acc;
          usc[(long long)kk * S] = uc;
          rc[(long long)kk * S] = res;
          bb += b * b;
          rr += res * res;
          um = uc;
          uc = up[t];
        }
      }
    }
  }
  const double s0 = block_sum(bb, sh);
  const double s1 = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    partial[2 * lb] = s0;
    partial[2 * lb + 1] = s1;
  }
}

// u = us + alpha p (with_p = 1: the last iteration's deferred update), u =
// (us + alpha2 p2) + alpha p (with_p = 2: the last two, p2 the older
// direction), or us (with_p = 0), written plane-major, and the true residual
// of that u:
// partial[2 lb] = sum (V f)^2, partial[2 lb + 1] = sum (V f - A u)^2.
// One block = 64 split slots with alternating colours (a red and a black
// column side by side are adjacent plane-major cells, so the plane-major
// accesses are coalesced too), one k-segment of four per wavefront.
template <bool C3 = false>
__device__ __forceinline__ void finish_body(Geo L, const double *__restrict__ tab,
                                            const double *__restrict__ vol,
                                            const double *__restrict__ f,
                                            const double *__restrict__ us,
                                            const double *__restrict__ p, double alpha,
                                            const double *__restrict__ p2, double alpha2, int with_p,
                                            double *__restrict__ u, double *__restrict__ partial,
                                            int lb, const double *__restrict__ tz3 = nullptr) {
  constexpr int NSEG = 4, U = 4;
  __shared__ double sh[4];
  const int sg = wave_id();
  const int slot = lb * kSegCols + (threadIdx.x & 63);
  const int c = slot & 1;
  const int m = slot >> 1;
  const bool valid = slot < 2 * L.H && m < (c ? L.ncol1 : L.ncol0);
  const int Ls = seg_len(L.nz, NSEG);
  const int k0 = min(sg * Ls, L.nz), k1 = min(k0 + Ls, L.nz);
  double bb = 0.0, rr = 0.0;
  if (valid && k1 > k0) {
    int i, j;
    col_ij(L, c, m, i, j);
    const Nbr nb = neighbours(L, i, j);
    const bool hx = L.has_x, hy = L.has_y;
    const long long S = L.S;
    const long long plane = (long long)L.nx * L.ny;
    const long long oc = (long long)j * L.nx + i;
    const long long oo = (long long)(1 - c) * L.cs, os = (long long)c * L.cs + m;
    const int nz = L.nz, P = L.P;
    auto val = [&](long long idx) -> double {
      if (!with_p) return us[idx];
      double v = us[idx];
      if (with_p == 2) v = v + alpha2 * p2[idx];
      return v + alpha * p[idx];
    };
    double uc = val(os + (long long)k0 * S);
    double um = k0 > 0 ? val(os + (long long)(k0 - 1) * S) : uc;
    int k = k0;
    for (; k < k1; k += U) {
      double up[U], uw[U], ue[U], usv[U], un[U], fv[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const int kk = min(k + t, k1 - 1);
        const long long o = (long long)kk * S;
        up[t] = val(os + (long long)min(kk + 1, nz - 1) * S);
        uw[t] = hx ? val(oo + nb.w + o) : 0.0;
        ue[t] = hx ? val(oo + nb.e + o) : 0.0;
        usv[t] = hy ? val(oo + nb.s + o) : 0.0;
        un[t] = hy ? val(oo + nb.n + o) : 0.0;
        fv[t] = f[(long long)kk * plane + oc];
      }
#pragma unroll
      for (int t = 0; t < U; ++t) {
        if (k + t < k1) {
          const int kk = k + t;
          double acc;
          if constexpr (C3) {
            const double *__restrict__ zc = tz3 + os;
            acc = op_row_v(tab, P, kk, hx, hy, zc[(long long)kk * S], kk + 1 < nz ? zc[(long long)(kk + 1) * S] : 0.0,
                           uc, um, up[t], uw[t], ue[t], usv[t], un[t]);
          } else {
            acc = op_row(tab, P, kk, hx, hy, uc, um, up[t], uw[t], ue[t], usv[t], un[t]);
          }
          const double b = vol[kk] * fv[t];
          const double res = b - acc;
          u[(long long)kk * plane + oc] = uc;
          bb += b * b;
          rr += res * res;
          um = uc;
          uc = up[t];
        }
      }
    }
  }
  const double s0 = block_sum(bb, sh);
  const double s1 = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    partial[2 * lb] = s0;
    partial[2 * lb + 1] = s1;
  }
}

template <bool C3 = false>
__global__ __launch_bounds__(kBlock) void k_begin(Geo L, const double *__restrict__ tab,
                                                  const double *__restrict__ vol,
                                                  const double *__restrict__ f,
                                                  const double *__restrict__ u0,
                                                  double *__restrict__ us, double *__restrict__ r,
                                                  double *__restrict__ partial,
                                                  const double *__restrict__ tz3 = nullptr) {
  begin_body<C3>(L, tab, vol, f, u0, us, r, partial, logical_block(), tz3);
}

template <bool C3 = false>
__global__ __launch_bounds__(kBlock) void k_finish(Geo L, const double *__restrict__ tab,
                                                   const double *__restrict__ vol,
                                                   const double *__restrict__ f,
                                                   const double *__restrict__ us,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ p2,
                                                   const PcgState *__restrict__ st, int with_p,
                                                   double *__restrict__ u, double *__restrict__ partial,
                                                   const double *__restrict__ tz3 = nullptr) {
  finish_body<C3>(L, tab, vol, f, us, p, with_p ? st->alpha : 0.0, p2, with_p == 2 ? st->alpha_prev : 0.0, with_p, u,
                  partial, logical_block(), tz3);
}

// The start and the end of a solve on the tiles of the CG operator step (a
// block: 32 m-columns by 16 rows, both colours, one k-segment of nseg; the
// horizontal neighbours of each level staged in a three-level LDS ring):
//   BEGIN:  us = u0 and r = V f - A u0 in the split layout, u0 and f
//           plane-major (src = u0, o1 = us, o2 = r);
//   !BEGIN: u = us + alpha p, (us + alpha2 p2) + alpha p or us (with_p = 1,
//           2, 0, as in finish_body) written plane-major, with the true
//           residual V f - A u of that u (src = us, o1 = u).
// partial[2 lb] = sum (V f)^2, partial[2 lb + 1] = sum res^2 over the block;
// blocks past the last segment write zeros.  Each cell's A u is formed in
// the order of op_row, so u and the residual equal the column kernels' (the
// block sums differ in their order).  WP: with_p as a compile-time constant
// (no branch per element).  smem: the block's LDS of kEndsSmem doubles, owned
// by the kernel so that several instantiations in one kernel share it.
constexpr int kEndsSmem = 3 * 2 * kTH * kTW + 4;
template <bool BEGIN, int WP = 0>
__device__ __forceinline__ void ends_tile_body(Geo L, int nseg, const double *__restrict__ tab,
                                               const double *__restrict__ vol,
                                               const double *__restrict__ f,
                                               const double *__restrict__ src,
                                               const double *__restrict__ p, double alpha,
                                               const double *__restrict__ p2, double alpha2,
                                               double *__restrict__ o1, double *__restrict__ o2,
                                               double *__restrict__ partial, int lb, double *smem) {
  double(*sp)[2][kTH][kTW] = reinterpret_cast<double(*)[2][kTH][kTW]>(smem);
  double *sh = smem + 3 * 2 * kTH * kTW;
  const int tiles_x = (L.hx2 + kTX - 1) / kTX;
  const int per_seg = tile_count(L.hx2, L.ny);
  const int sg = lb / per_seg, tt = lb - sg * per_seg;
  const int ty = tt / tiles_x, tx = tt - ty * tiles_x;
  const int Ls = seg_len(L.nz, nseg);
  const int k0 = min(sg * Ls, L.nz), k1 = min(k0 + Ls, L.nz);
  double bb = 0.0, rs = 0.0;
  if (k1 > k0) {
    const int t = threadIdx.x;
    const int mx0 = tx * kTX, j0 = ty * kTY;
    const int nxm = min(kTX, L.hx2 - mx0);
    const int nyr = min(kTY, L.ny - j0);
    const int x = t & 31, r0 = t >> 5;  // own cells: rows r0 and r0 + 8, both colours
    const long long S = L.S, cs = L.cs, plane = (long long)L.nx * L.ny;
    long long off[4], pmo[4];  // split and plane-major offsets at level 0
    bool ok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = e & 1, rr = r0 + 8 * (e >> 1), j = j0 + rr;
      ok[e] = x < nxm && rr < nyr;
      off[e] = (long long)c * cs + (long long)j * L.hx2 + mx0 + x;
      pmo[e] = (long long)j * L.nx + 2 * (mx0 + x) + ((j + c) & 1);
    }
    // one halo cell per thread for threads 0..159 (rows below / above the
    // tile, both colours; then the cells left / right of each row), with its
    // offset in the layout src is read in
    bool hok = false;
    long long hoff = 0;
    int hc = 0, hr = 0, hx = 0;
    if (t < 128) {
      const int side = t >> 6, c = (t >> 5) & 1, xx = t & 31;
      const int j = side ? wrapi(j0 + nyr, L.ny) : wrapi(j0 - 1, L.ny);
      hok = xx < nxm;
      hoff = BEGIN ? (long long)j * L.nx + 2 * (mx0 + xx) + ((j + c) & 1)
                   : (long long)c * cs + (long long)j * L.hx2 + mx0 + xx;
      hc = c;
      hr = side ? nyr + 1 : 0;
      hx = xx + 1;
    } else if (t < 160) {
      const int side = (t - 128) >> 4, rr = (t - 128) & 15;
      const int j = j0 + rr;
      const int i = side ? wrapi(2 * (mx0 + nxm), L.nx) : wrapi(2 * mx0 - 1, L.nx);
      const int c = (i + j) & 1;
      hok = rr < nyr;
      hoff = BEGIN ? (long long)j * L.nx + i : (long long)c * cs + (long long)j * L.hx2 + (i >> 1);
      hc = c;
      hr = rr + 1;
      hx = side ? nxm + 1 : 0;
    }
    const long long lstride = BEGIN ? plane : S;  // level stride of src
    auto val = [&](long long idx) -> double {
      if constexpr (BEGIN || WP == 0) {
        return src[idx];
      } else {
        double v = src[idx];
        if constexpr (WP == 2) v = v + alpha2 * p2[idx];
        return v + alpha * p[idx];
      }
    };
    // level k: own values into v (and LDS buffer b when b >= 0)
    auto level = [&](int k, int b, double *v) {
      const long long o = (long long)k * lstride;
      double w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) w[e] = ok[e] ? val((BEGIN ? pmo[e] : off[e]) + o) : 0.0;
      double hv = 0.0;
      if (b >= 0 && hok) hv = val(hoff + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = w[e];
        if (b >= 0 && ok[e]) sp[b][e & 1][r0 + 8 * (e >> 1) + 1][x + 1] = w[e];
      }
      if (b >= 0 && hok) sp[b][hc][hr][hx] = hv;
    };
    const double *__restrict__ tv = tab + TV * L.P;
    const double *__restrict__ txv = tab + TX * L.P;
    const double *__restrict__ tyv = tab + TY * L.P;
    const double *__restrict__ tz = tab + TZ * L.P;
    double pm[4], pc[4], pn[4];
    level(k0, k0 % 3, pc);
    if (k0 > 0) level(k0 - 1, -1, pm);
    else {
#pragma unroll
      for (int e = 0; e < 4; ++e) pm[e] = pc[e];
    }
    for (int k = k0; k < k1; ++k) {
      if (k + 1 < k1) level(k + 1, (k + 1) % 3, pn);
      else if (k + 1 < L.nz) level(k + 1, -1, pn);
      else {
#pragma unroll
        for (int e = 0; e < 4; ++e) pn[e] = pc[e];
      }
      double fv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) fv[e] = ok[e] ? __builtin_nontemporal_load(&f[(long long)k * plane + pmo[e]]) : 0.0;
      __syncthreads();
      const int b = k % 3;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (ok[e]) {
          const int c = e & 1, rr = r0 + 8 * (e >> 1);
          const int par = (j0 + rr + c) & 1;  // 1: the cell sits at an odd i
          const double(*oth)[kTW] = sp[b][1 - c];
          const double pw = oth[rr + 1][x + par];
          const double pe = oth[rr + 1][x + 1 + par];
          const double ps = oth[rr][x + 1];
          const double pnn = oth[rr + 2][x + 1];
          const double pcv = pc[e];
          double acc = tv[k] * pcv;
          acc = acc + txv[k] * (pcv - pw);
          acc = acc + txv[k] * (pcv - pe);
          acc = acc + tyv[k] * (pcv - ps);
          acc = acc + tyv[k] * (pcv - pnn);
          acc = acc + tz[k] * (pcv - pm[e]);
          acc = acc + tz[k + 1] * (pcv - pn[e]);
          const double bv = vol[k] * fv[e];
          const double res = bv - acc;
          if constexpr (BEGIN) {
            __builtin_nontemporal_store(pcv, &o1[off[e] + (long long)k * S]);
            __builtin_nontemporal_store(res, &o2[off[e] + (long long)k * S]);
          } else {
            // plain store: a row's two colours interleave in u, so each store
            // fills every other double of its lines and the L2 merges the
            // halves (streaming stores measured 1.67x the written bytes)
            o1[pmo[e] + (long long)k * plane] = pcv;
          }
          bb += bv * bv;
          rs += res * res;
        }
        pm[e] = pc[e];
        pc[e] = pn[e];
      }
    }
  }
  const double s0 = block_sum(bb, sh);
  const double s1 = block_sum(rs, sh);
  if (threadIdx.x == 0) {
    partial[2 * lb] = s0;
    partial[2 * lb + 1] = s1;
  }
}

__global__ __launch_bounds__(kBlock) void k_begin_tile(Geo L, int nseg, const double *__restrict__ tab,
                                                       const double *__restrict__ vol,
                                                       const double *__restrict__ f,
                                                       const double *__restrict__ u0, double *__restrict__ us,
                                                       double *__restrict__ r, double *__restrict__ partial) {
  __shared__ double smem[kEndsSmem];
  ends_tile_body<true>(L, nseg, tab, vol, f, u0, nullptr, 0.0, nullptr, 0.0, us, r, partial, logical_block(), smem);
}

template <int WP>
__global__ __launch_bounds__(kBlock) void k_finish_tile(Geo L, int nseg, const double *__restrict__ tab,
                                                        const double *__restrict__ vol,
                                                        const double *__restrict__ f,
                                                        const double *__restrict__ us,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ p2,
                                                        const PcgState *__restrict__ st,
                                                        double *__restrict__ u, double *__restrict__ partial) {
  __shared__ double smem[kEndsSmem];
  ends_tile_body<false, WP>(L, nseg, tab, vol, f, us, p, WP ? st->alpha : 0.0, p2, WP == 2 ? st->alpha_prev : 0.0, u,
                            nullptr, partial, logical_block(), smem);
}

// -------------------------------------------------------------------------
// CG vector kernels (FP64, flat over the split vectors; padding entries stay
// zero).  Each block writes its partial sums; k_finalize reduces them in a
// fixed order, so every result is independent of scheduling.
// -------------------------------------------------------------------------

template <typename Z> struct Vec2;
template <> struct Vec2<double> { using T = double2; };
template <> struct Vec2<float> { using T = float2; };

// partial sums of <r, z> and <z, q>
template <typename Z>
__device__ __forceinline__ void dots_body(const double2 *__restrict__ r,
                                                 const typename Vec2<Z>::T *__restrict__ z,
                                                 const double2 *__restrict__ q, long long n2,
                                                 const PcgState *__restrict__ st,
                                                 double *__restrict__ partial, int lb, int nblocks) {
  __shared__ double sh[4];
  if (st->done) return;
  const long long t = (long long)lb * kBlock + threadIdx.x;
  const long long stride = (long long)nblocks * kBlock;
  double rz = 0.0, zq = 0.0;
  if (st->flexible) {
    for (long long e = t; e < n2; e += stride) {
      const double2 rv = ld_nt(&r[e]), qv = ld_nt(&q[e]);
      const auto zv = z[e];
      const double zx = (double)zv.x, zy = (double)zv.y;
      rz += rv.x * zx + rv.y * zy;
      zq += zx * qv.x + zy * qv.y;
    }
  } else {  // the classic beta needs <r, z> only
    for (long long e = t; e < n2; e += stride) {
      const double2 rv = ld_nt(&r[e]);
      const auto zv = z[e];
      rz += rv.x * (double)zv.x + rv.y * (double)zv.y;
    }
  }
  const double s0 = block_sum(rz, sh);
  const double s1 = block_sum(zq, sh);
  if (threadIdx.x == 0) {
    partial[2 * lb] = s0;
    partial[2 * lb + 1] = s1;
  }
}

template <typename Z>
__global__ __launch_bounds__(kBlock) void k_dots(const double2 *__restrict__ r,
                                                 const typename Vec2<Z>::T *__restrict__ z,
                                                 const double2 *__restrict__ q, long long n2,
                                                 const PcgState *__restrict__ st,
                                                 double *__restrict__ partial) {
  dots_body<Z>(r, z, q, n2, st, partial, logical_block(), gridDim.x);
}

// F_CONV_PENDING: F_CONV if a residual update is pending, else nothing (a
// batched grid's first step has no update before its V-cycle).
enum FinalizeMode : int {
  F_INIT = 0, F_KAPPA = 1, F_ALPHA = 2, F_CONV = 3, F_BETA = 4, F_TRUE = 5, F_UNIT = 6, F_CONV_PENDING = 7
};

// One block: reduce nq interleaved partial sums over nblk blocks in a fixed
// order and advance the CG scalars (Appendix B, Alg. PCG).
__device__ __forceinline__ void finalize_body(const double *__restrict__ partial, int nblk,
                                                     int nq, PcgState *__restrict__ st, int mode,
                                                     double rtol, double atol, int rel_to_rhs, int lb, int nblocks) {
  __shared__ double sh[4];
  __shared__ double tot[2];
  if (mode != F_TRUE && mode != F_INIT && st->done) return;
  if (mode == F_CONV_PENDING) {
    if (!st->pending) return;
    mode = F_CONV;
  }
  // nq <= 2.  Each thread adds the blocks threadIdx.x + i kBlock in order of
  // i; eight of them are loaded before the first is added, so the latency of
  // the loads (written by other XCDs) is paid once per eight.
  double v[2] = {0.0, 0.0};
  for (int b0 = threadIdx.x; b0 < nblk; b0 += 8 * kBlock) {
    double a[8][2];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int b = b0 + t * kBlock;
#pragma unroll
      for (int qi = 0; qi < 2; ++qi) a[t][qi] = (b < nblk && qi < nq) ? partial[(long long)b * nq + qi] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
#pragma unroll
      for (int qi = 0; qi < 2; ++qi) v[qi] = b0 + t * kBlock < nblk ? v[qi] + a[t][qi] : v[qi];
    }
  }
  for (int qi = 0; qi < nq; ++qi) {
    const double s = block_sum(v[qi], sh);
    if (threadIdx.x == 0) tot[qi] = s;
  }
  if (threadIdx.x != 0) return;
  switch (mode) {
    case F_INIT: {
      const double bn = sqrt(tot[0]), r0 = sqrt(tot[1]);
      st->b_norm = bn;
      st->r0_norm = r0;
      st->r_norm = r0;
      const double ref = rel_to_rhs ? bn : r0;
      const double th = fmax(rtol * ref, atol);
      st->thresh = th;
      st->iter = 0;
      st->pending = 0;
      st->alpha = st->alpha_prev = st->beta = st->kappa_old = 0.0;
      if (!isfinite(r0) || !isfinite(bn)) {
        st->done = 1;
        st->status = -4;
      } else if (r0 == 0.0 || r0 < th) {
        st->done = 1;
        st->status = 0;
      } else if (st->maxiter <= 0) {
        st->done = 1;
        st->status = 1;
      } else {
        st->done = 0;
        st->status = 1;
      }
      break;
    }
    case F_KAPPA:
      st->kappa_old = tot[0];
      if (!isfinite(tot[0])) { st->done = 1; st->status = -4; }
      break;
    case F_ALPHA: {
      const double a = st->kappa_old / tot[0];
      st->alpha_prev = st->alpha;
      st->alpha = a;
      st->pending = 1;
      if (!isfinite(a)) { st->done = 1; st->status = -4; }
      break;
    }
    case F_CONV: {
      const double rn = sqrt(tot[0]);
      st->r_norm = rn;
      st->iter += 1;
      st->pending = 0;
      if (!isfinite(rn)) { st->done = 1; st->status = -4; }
      else if (rn < st->thresh) { st->done = 1; st->status = 0; }
      else if (st->iter >= st->maxiter) { st->done = 1; st->status = 1; }
      break;
    }
    case F_BETA: {
      const double kappa = tot[0];
      if (st->iter == 0) {  // first preconditioned residual: kappa_0 = <r_0, z_0>
        st->kappa_old = kappa;
        if (!isfinite(kappa)) { st->done = 1; st->status = -4; }
        break;
      }
      const double beta = st->flexible ? -st->alpha * tot[1] / st->kappa_old : kappa / st->kappa_old;
      st->beta = beta;
      st->kappa_old = kappa;
      if (!isfinite(beta)) { st->done = 1; st->status = -4; }
      break;
    }
    case F_UNIT:  // stand-alone multigrid: unit steps along z, no direction memory
      st->alpha = 1.0;
      st->alpha_prev = 1.0;
      st->beta = 0.0;
      break;
    case F_TRUE:  // partials of k_finish: [||V f||^2, ||V f - A u||^2]
      st->true_r_norm = sqrt(tot[nq - 1]);
      break;
  }
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partial, int nblk,
                                                     int nq, PcgState *__restrict__ st, int mode,
                                                     double rtol, double atol, int rel_to_rhs) {
  finalize_body(partial, nblk, nq, st, mode, rtol, atol, rel_to_rhs, logical_block(), gridDim.x);
}

// -------------------------------------------------------------------------
// The coarsest level's sweeps in one cooperative launch (every block
// resident): nu_coarse red/black pairs from u = 0, the half-sweeps separated
// by a grid-wide barrier.  Each half-sweep is the device body the per-sweep
// kernels run, with the same template arguments (the first one the zero-start
// segmented sweep, the others the LDS-tiled one in FP64 or the segmented one
// in FP32), so the values are those of the separate launches; the block index
// of each body comes from the same XCD-contiguous map.
//
// grid_barrier: sense-reversing over bar[0] (arrivals) and bar[1]
// (generation), zeroed once when the grid is created; the last block to
// arrive resets the count and advances the generation.  Agent-scope fences
// release a block's writes before it arrives and acquire the others' after it
// leaves (the XCDs' L2 caches are not coherent with each other).  The wait is
// bounded: a block that polls kBarrierSpins times without the generation
// moving gives up, raises bar[2] and leaves, so the kernel always ends.
// -------------------------------------------------------------------------
constexpr long kBarrierSpins = 1L << 24;

// One release fence before a block arrives and one acquire fence after it
// leaves; the arrival and the polling are relaxed (an acquiring poll would
// invalidate the L2 on every read).  The last block to arrive acquires the
// others' writes before it releases the new generation.
__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kBarrierSpins) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// NSEG: the level's k-segments (8 or 16); SEG: the segmented sweep's register
// depth, TSEG the tiled one's (as the per-sweep dispatch picks them).
template <typename R, int NSEG, int SEG, int TSEG>
__global__ __launch_bounds__(NSEG * 64) void k_coarse_sweeps(Geo L, const R *__restrict__ tab,
                                                             const R *__restrict__ b, R *__restrict__ u,
                                                             int sweeps, const int *__restrict__ done,
                                                             unsigned *__restrict__ bar) {
  if (is_done(done)) return;  // the flag does not change during the launch: every block leaves
  const int g8 = gridDim.x >> 3;
  const int lb0 = (blockIdx.x & 7) * g8 + (blockIdx.x >> 3);
  const long long cs = L.cs;
  const int nb0 = (L.ncol0 + kSegCols - 1) / kSegCols, nb1 = (L.ncol1 + kSegCols - 1) / kSegCols;
  const int ntiles = ((L.hx2 + kSTX - 1) / kSTX) * (L.ny / 2);
  for (int it = 0; it < sweeps; ++it) {
    for (int c = 0; c < 2; ++c) {
      const R *bo = b + (long long)c * cs;
      const R *uo = u + (long long)(1 - c) * cs;
      R *own = u + (long long)c * cs;
      if (it == 0 && c == 0) {
        for (int lb = lb0; lb < nb0; lb += gridDim.x) {
          smooth_seg_body<R, true, true, false, SEG, NSEG, R>(L, tab, 0, bo, uo, own, R(1), done, lb, nb0);
          __syncthreads();
        }
      } else if constexpr (std::is_same<R, double>::value) {
        for (int lb = lb0; lb < ntiles; lb += gridDim.x) {
          smooth_tile_body<TSEG, NSEG, false>(L, tab, c, bo, uo, own, done, lb);
          __syncthreads();
        }
      } else {
        const int nb = c ? nb1 : nb0;
        for (int lb = lb0; lb < nb; lb += gridDim.x) {
          smooth_seg_body<R, false, true, false, SEG, NSEG, R>(L, tab, c, bo, uo, own, R(1), done, lb, nb);
          __syncthreads();
        }
      }
      if (it + 1 < sweeps || c == 0) grid_barrier(bar, gridDim.x);
    }
  }
}

// -------------------------------------------------------------------------
// Grid-free operator application (no device allocation): a coefficient table
// is written into a caller-provided device area from kernel arguments, a
// chunk per launch (the arguments are copied at launch, so nothing on the host
// has to outlive the call), and y = A x is evaluated straight in the
// plane-major layout idx = (k*ny + j)*nx + i.
// -------------------------------------------------------------------------
constexpr int kTabChunk = 256;
struct TabChunk {
  int off, n;
  double v[kTabChunk];
};

__global__ __launch_bounds__(kBlock) void k_put_table(double *__restrict__ dst, TabChunk c) {
  for (int t = threadIdx.x; t < c.n; t += kBlock) dst[c.off + t] = c.v[t];
}

// One lane per column, blockIdx.y the k-segment (of nseg).  tab: V, Tx, Ty, Tz
// in slots of nz+1 (the TV..TZ slots of a level table).  Each cell is the
// same expression, in the same order, as in k_apply.
__global__ __launch_bounds__(kBlock) void k_apply_nat(int nx, int ny, int nz, int nseg,
                                                      const double *__restrict__ tab,
                                                      const double *__restrict__ x,
                                                      double *__restrict__ y) {
  const long long plane = (long long)nx * ny;
  const long long col = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (col >= plane) return;
  const int Ls = seg_len(nz, nseg);
  const int k0 = min((int)blockIdx.y * Ls, nz), k1 = min(k0 + Ls, nz);
  if (k0 >= k1) return;
  const int i = (int)(col % nx), j = (int)(col / nx);
  const bool hx = nx > 1, hy = ny > 1;
  const long long cw = (long long)j * nx + wrapi(i - 1, nx), ce = (long long)j * nx + wrapi(i + 1, nx);
  const long long cs = (long long)wrapi(j - 1, ny) * nx + i, cn = (long long)wrapi(j + 1, ny) * nx + i;
  const int P = nz + 1;
  const double *__restrict__ tv = tab + TV * P;
  const double *__restrict__ tx = tab + TX * P;
  const double *__restrict__ ty = tab + TY * P;
  const double *__restrict__ tz = tab + TZ * P;
  auto cell = [&](int k, double xc, double xm, double xp, double w, double e, double so, double no) {
    double acc = tv[k] * xc;
    if (hx) {
      acc = acc + tx[k] * (xc - w);
      acc = acc + tx[k] * (xc - e);
    }
    if (hy) {
      acc = acc + ty[k] * (xc - so);
      acc = acc + ty[k] * (xc - no);
    }
    acc = acc + tz[k] * (xc - xm);
    acc = acc + tz[k + 1] * (xc - xp);
    return acc;
  };
  double xc = x[(long long)k0 * plane + col];
  double xm = k0 > 0 ? x[(long long)(k0 - 1) * plane + col] : xc;
  int k = k0;
  for (; k + kChunk <= k1; k += kChunk) {
    double xp[kChunk], w[kChunk], e[kChunk], so[kChunk], no[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      const long long o = (long long)(k + t) * plane;
      xp[t] = x[(long long)min(k + t + 1, nz - 1) * plane + col];
      w[t] = hx ? x[o + cw] : 0.0;
      e[t] = hx ? x[o + ce] : 0.0;
      so[t] = hy ? x[o + cs] : 0.0;
      no[t] = hy ? x[o + cn] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      y[(long long)(k + t) * plane + col] = cell(k + t, xc, xm, xp[t], w[t], e[t], so[t], no[t]);
      xm = xc;
      xc = xp[t];
    }
  }
  for (; k < k1; ++k) {
    const long long o = (long long)k * plane;
    const double xpv = x[(long long)min(k + 1, nz - 1) * plane + col];
    y[o + col] = cell(k, xc, xm, xpv, hx ? x[o + cw] : 0.0, hx ? x[o + ce] : 0.0, hy ? x[o + cs] : 0.0,
                      hy ? x[o + cn] : 0.0);
    xm = xc;
    xc = xpv;
  }
}

}  // namespace ell
