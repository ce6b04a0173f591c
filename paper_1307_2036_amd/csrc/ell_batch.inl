// Batch engine: many solves of uneven size advanced together.
//
// Every stage of a CG iteration (the fused operator step, the residual
// update, each V-cycle half-sweep / restriction / prolongation, the dots and
// the scalar updates) is one grouped launch covering every active grid: a
// block looks up its grid in a stage table (a ballot over the entries' first
// blocks)
// and runs the same device body as the single-grid kernel on that grid's
// arrays.  Grids of different depth share the launches of the levels they
// have; each grid carries its own CG state on the device, so converged grids
// drop out (their blocks return at once) while the others continue.  A host
// worker thread admits new requests and retires finished ones between
// iterations, so requests that arrive while others run join the next
// iteration (continuous batching) and their work overlaps on the device.
//
// Included into ell.hip (it uses that file's launch helpers and grid type).

#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace ellb {  // named: the kernels keep external symbols (named in profiles)

constexpr int kMaxLevels = 16;

struct LevelDev {
  Geo geo;
  const void *tab;
  void *b;
  void *u;
};

// Everything the batched kernels need of one grid (device copy).
struct GridDev {
  LevelDev lev[kMaxLevels];
  const double *tab64_0;
  const double *vol0;  // finest-level cell volumes
  double *us, *r, *z, *p, *p2, *p3, *q;  // p_K in {p, p2, p3}[dir_slot(K)]
  float *u32;
  double *partial;
  PcgState *st;
  long long n2;
  int L, nb_apply, nb_flat, prolong;
  int nb_begin, nb_finish;  // blocks of the start / end kernels (partial sums each)
  int ends_tile, ends_nseg;  // start / end on the operator step's LDS tiles, their k-segments
  int apply_tile, apply_nseg;  // CG operator step: LDS-tiled kernel and its k-segments
  int nb_tiles;                // finest level: tiles of a tiled half-sweep (0: column kernel)
  int nb_dot;                  // partial sums of the fused CG dots (0: separate dot pass)
  int nb_upd0, nb_upd;         // fused residual update: colour-0 slots, all slots (0: separate pass)
};

struct StageEnt {
  const GridDev *g;
  int block0;
  int aux;  // start / end tables: index of the request record
};

// What the start and end of one solve need beyond its grid: the caller's
// vectors and the stopping rule.
struct ReqDev {
  const double *f;
  double *u;
  double rtol, atol;
  int rel_to_rhs, maxiter, flexible, pad;
};

enum Role : int { ROLE_COARSE = 0, ROLE_FINE64 = 1, ROLE_PRE32 = 2 };

__device__ __forceinline__ int ui(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ long long ull(long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ Geo ugeo(const Geo &g) {
  Geo r;
  r.nx = ui(g.nx);
  r.ny = ui(g.ny);
  r.nz = ui(g.nz);
  r.H = ui(g.H);
  r.ncol0 = ui(g.ncol0);
  r.ncol1 = ui(g.ncol1);
  r.hx2 = ui(g.hx2);
  r.has_x = ui(g.has_x);
  r.has_y = ui(g.has_y);
  r.P = ui(g.P);
  r.S = ui(g.S);
  r.nseg = ui(g.nseg);
  r.cs = ull(g.cs);
  return r;
}

// The entry whose block range holds block b (b wave-uniform, every lane
// active): the entries are sorted by their first block, so the number of
// entries that start at or before b is the index plus one.  Each lane tests
// one entry, 64 at a time (one vector load and a ballot per 64 entries, where
// a binary search waited for log2(n) dependent loads).
__device__ __forceinline__ int find_ent(const StageEnt *e, int n, int b) {
  const int lane = threadIdx.x & 63;
  int cnt = 0;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    const bool p = i < n && e[i].block0 <= b;
    const unsigned long long m = __ballot(p);
    cnt += __popcll(m);
    if (m != ~0ull) break;  // the first entry past b lies in this chunk
  }
  return ui(cnt - 1);
}

// R: arithmetic type; TB: type of b.  ROLE selects the arrays of the stage.
template <typename R, bool ZERO, bool FINE, int SEG, typename TB, int ROLE, int NSEG = 4>
__global__ __launch_bounds__(NSEG * 64) void kb_smooth(const StageEnt *__restrict__ ents, int nent, int total,
                                                       int l, int c) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const LevelDev &Lv = gd->lev[l];
  const Geo G = ugeo(Lv.geo);
  const R *tab;
  const TB *b;
  R *u;
  if (ROLE == ROLE_FINE64) {
    tab = (const R *)gd->tab64_0;
    b = (const TB *)gd->r;
    u = (R *)gd->z;
  } else if (ROLE == ROLE_PRE32) {
    tab = (const R *)Lv.tab;
    b = (const TB *)gd->r;
    u = (R *)gd->u32;
  } else {
    tab = (const R *)Lv.tab;
    b = (const TB *)Lv.b;
    u = (R *)Lv.u;
  }
  tab = cp(tab);
  b = gp(b);
  u = gp(u);
  smooth_seg_body<R, ZERO, true, FINE, SEG, NSEG, TB>(G, tab, c, b + (long long)c * G.cs,
                                                   u + (long long)(1 - c) * G.cs, u + (long long)c * G.cs,
                                                   R(1), gp(&gd->st->done), ui(bg - ents[e].block0), 0);
}

// The finest level's FP64 half-sweep of the grids that take the LDS-tiled
// kernel (NSEG k-segments, one block per tile); with DOT (the last two
// post-smoothing half-sweeps) also the partial sums <r, z> and <z, q> of the
// fused CG dots (colour 1 into the first nb_tiles pairs, colour 0 after them).
template <int SEG, int NSEG, bool DOT>
__global__ __launch_bounds__(NSEG * 64) void kb_smooth_tile(const StageEnt *__restrict__ ents, int nent, int total,
                                                            int c) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const Geo G = ugeo(gd->lev[0].geo);
  const double *tab = cp(gd->tab64_0);
  const double *b = gp(gd->r);
  double *u = gp(gd->z);
  const long long cs = G.cs;
  smooth_tile_body<SEG, NSEG, true, DOT ? 2 : 0>(G, tab, c, b + c * cs, u + (1 - c) * cs, u + c * cs,
                                              gp(&gd->st->done), ui(bg - ents[e].block0), gp(gd->partial),
                                              c == 1 ? 0 : ui(gd->nb_tiles), gp(gd->q) + c * cs);
}

// The mixed-precision V-cycle's finest colour-1 post-smoothing sweep (FP64)
// with the last prolongation applied on the fly, as k_smooth_tile_pro32: the
// FP32 colour-0 values of u32 and the FP32 coarse correction are staged, the
// correction formed in FP32 and added in FP64 (the values the prolongation
// pass would write into z); DOT as kb_smooth_tile.  PAIR: every grid of the
// stage has the coarse layout of paired loads (pro32_pairs_ok), else the
// coarse values load one by one.
template <int SEG, int NSEG, bool DOT, bool PAIR>
__global__ __launch_bounds__(NSEG * 64) void kb_smooth_tile_pro32(const StageEnt *__restrict__ ents, int nent,
                                                                  int total) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const Geo G = ugeo(gd->lev[0].geo);
  const Geo C = ugeo(gd->lev[1].geo);
  const long long cs = G.cs;
  smooth_tile_body<SEG, NSEG, true, DOT ? 2 : 0, false, true, 4, PAIR, float>(
      G, cp(gd->tab64_0), 1, gp(gd->r) + cs, gp((const float *)gd->u32), gp(gd->z) + cs, gp(&gd->st->done),
      ui(bg - ents[e].block0), gp(gd->partial), 0, gp(gd->q) + cs, nullptr, nullptr, &C,
      gp((const float *)gd->lev[1].u));
}

// The finest level's first pre-smoothing pair of the grids with the fused
// residual update (column kernel; ROLE_PRE32: the FP32 sweep of the
// mixed-precision V-cycle, ROLE_FINE64: FP64).  HEAD: at the start of a
// grid's first step (nothing pending, no iteration yet), the plain pair;
// otherwise (the end of every step, after alpha): the pair with r -= alpha q,
// whose convergence test ends the step and whose V-cycle the next step
// continues.  A block whose grid does not take this form of the pair returns
// at once.
template <typename R, bool ZERO, int SEG, int NSEG, int ROLE, bool HEAD>
__global__ __launch_bounds__(NSEG * 64) void kb_smooth_upd(const StageEnt *__restrict__ ents, int nent, int total,
                                                           int c) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const PcgState *st = gp(gd->st);
  const int pending = ui(st->pending);
  if (HEAD ? (pending != 0 || ui(st->iter) != 0) : pending == 0) return;
  const Geo G = ugeo(gd->lev[0].geo);
  const R *tab = cp(ROLE == ROLE_FINE64 ? (const R *)gd->tab64_0 : (const R *)gd->lev[0].tab);
  double *r = gp(gd->r);
  R *u = gp(ROLE == ROLE_FINE64 ? (R *)gd->z : (R *)gd->u32);
  const long long cs = G.cs;
  const int lb = ui(bg - ents[e].block0);
  if (HEAD)
    smooth_seg_body<R, ZERO, true, true, SEG, NSEG, double>(G, tab, c, r + c * cs, u + (1 - c) * cs, u + c * cs,
                                                            R(1), &st->done, lb, 0);
  else
    smooth_seg_body<R, ZERO, true, true, SEG, NSEG, double, true>(
        G, tab, c, r + c * cs, u + (1 - c) * cs, u + c * cs, R(1), &st->done, lb, 0, r + c * cs,
        gp(gd->q) + c * cs, st, gp(gd->partial), c == 1 ? ui(gd->nb_upd0) : 0);
}

// Colour 1 of that pair on the tiled kernel (FP64 batches).
template <int SEG, int NSEG, bool HEAD>
__global__ __launch_bounds__(NSEG * 64) void kb_smooth_tile_upd(const StageEnt *__restrict__ ents, int nent,
                                                                int total) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const PcgState *st = gp(gd->st);
  const int pending = ui(st->pending);
  if (HEAD ? (pending != 0 || ui(st->iter) != 0) : pending == 0) return;
  const Geo G = ugeo(gd->lev[0].geo);
  double *r = gp(gd->r);
  double *u = gp(gd->z);
  const long long cs = G.cs;
  const int lb = ui(bg - ents[e].block0);
  if (HEAD)
    smooth_tile_body<SEG, NSEG, true>(G, cp(gd->tab64_0), 1, r + cs, u, u + cs, &st->done, lb);
  else
    smooth_tile_body<SEG, NSEG, true, 0, true>(G, cp(gd->tab64_0), 1, r + cs, u, u + cs, &st->done, lb,
                                               gp(gd->partial), ui(gd->nb_upd0), gp(gd->q) + cs, r + cs, st);
}

template <typename R, typename TB, int ROLE>
__global__ __launch_bounds__(kBlock) void kb_restrict(const StageEnt *__restrict__ ents, int nent, int total,
                                                      int l) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const LevelDev &F = gd->lev[l];
  const LevelDev &C = gd->lev[l + 1];
  const TB *b = ROLE == ROLE_COARSE ? (const TB *)F.b : (const TB *)gd->r;
  const R *u = ROLE == ROLE_COARSE ? (const R *)F.u : (ROLE == ROLE_PRE32 ? (const R *)gd->u32 : (const R *)gd->z);
  resid_restrict_bz_body<R, TB>(ugeo(F.geo), ugeo(C.geo), cp((const R *)F.tab), gp(b), gp(u), gp((R *)C.b),
                                gp(&gd->st->done), ui(bg - ents[e].block0), 0);
}

template <typename R, int MODE, int ROLE>
__global__ __launch_bounds__(kBlock) void kb_prolong(const StageEnt *__restrict__ ents, int nent, int total,
                                                     int l) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const LevelDev &F = gd->lev[l];
  const LevelDev &C = gd->lev[l + 1];
  R *u = ROLE == ROLE_FINE64 ? (R *)gd->z : (R *)F.u;
  prolong_body<R, true, MODE>(ugeo(F.geo), ugeo(C.geo), gp((const R *)C.u), gp(u), gp(&gd->st->done),
                              ui(bg - ents[e].block0), 0);
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void kb_prolong_out(const StageEnt *__restrict__ ents, int nent,
                                                         int total) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  prolong_out_body<float, double, MODE>(ugeo(gd->lev[0].geo), ugeo(gd->lev[1].geo), gp((const float *)gd->lev[1].u),
                                        gp(gd->u32), gp(gd->z), gp(&gd->st->done), ui(bg - ents[e].block0), 0);
}

// The colour-0 bilinear prolongation of the grids that take the LDS-tiled
// kernel (one block per tile of level l), in place or, OUT, from the FP32
// finest level into the FP64 output z (the mixed-precision V-cycle).
template <typename R, int ROLE>
__global__ __launch_bounds__(kBlock) void kb_prolong_tile(const StageEnt *__restrict__ ents, int nent, int total,
                                                          int l) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const LevelDev &F = gd->lev[l];
  const LevelDev &C = gd->lev[l + 1];
  R *u = gp(ROLE == ROLE_FINE64 ? (R *)gd->z : (R *)F.u);
  prolong_tile_body<R, kSeg>(ugeo(F.geo), ugeo(C.geo), gp((const R *)C.u), u, gp(&gd->st->done),
                             ui(bg - ents[e].block0));
}

__global__ __launch_bounds__(kBlock) void kb_prolong_out_tile(const StageEnt *__restrict__ ents, int nent,
                                                              int total) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  prolong_tile_body<float, kSeg, double>(ugeo(gd->lev[0].geo), ugeo(gd->lev[1].geo),
                                         gp((const float *)gd->lev[1].u), gp(gd->u32), gp(&gd->st->done),
                                         ui(bg - ents[e].block0), gp(gd->z));
}

// The search direction of iteration K of a grid.
__device__ __forceinline__ double *dir_dev(const GridDev *gd, int K) {
  const int i = dir_slot(K);
  return i == 0 ? gd->p : (i == 1 ? gd->p2 : gd->p3);
}

__global__ __launch_bounds__(kBlock) void kb_apply_dir(const StageEnt *__restrict__ ents, int nent, int total) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const PcgState *st = gp(gd->st);
  const int K = ui(st->iter) + 1;  // iteration about to run
  double *pold = gp(dir_dev(gd, K - 1));
  double *pold2 = gp(dir_dev(gd, K - 2));
  double *pnew = gp(dir_dev(gd, K));
  if (ui(gd->apply_tile))
    apply_dir_tile_body<double>(ugeo(gd->lev[0].geo), ui(gd->apply_nseg), cp(gd->tab64_0), gp(gd->z), pold, pold2,
                                pnew, gp(gd->q), gp(gd->us), st, K == 1 ? 1 : 0, deferred_updates(K),
                                gp(gd->partial), ui(bg - ents[e].block0));
  else
    apply_dir_body<double, 1>(ugeo(gd->lev[0].geo), cp(gd->tab64_0), gp(gd->z), pold, pold2, pnew, gp(gd->q),
                              gp(gd->us), st, K == 1 ? 1 : 0, deferred_updates(K), gp(gd->partial),
                              ui(bg - ents[e].block0), 0);
}

__global__ __launch_bounds__(kBlock) void kb_update_r(const StageEnt *__restrict__ ents, int nent, int total) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  update_r_body(gp((double2 *)gd->r), gp((const double2 *)gd->q), ull(gd->n2), gp(gd->st), gp(gd->partial),
                ui(bg - ents[e].block0), ui(gd->nb_flat));
}

__global__ __launch_bounds__(kBlock) void kb_dots(const StageEnt *__restrict__ ents, int nent, int total) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  dots_body<double>(gp((const double2 *)gd->r), gp((const double2 *)gd->z), gp((const double2 *)gd->q),
                    ull(gd->n2), gp(gd->st), gp(gd->partial), ui(bg - ents[e].block0), ui(gd->nb_flat));
}

// Start of the solves of a table: split-layout u and r = V f - A u0.
__global__ __launch_bounds__(kBlock) void kb_begin(const StageEnt *__restrict__ ents, int nent, int total,
                                                   const ReqDev *__restrict__ reqs) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const ReqDev *rq = gp(reqs + ents[e].aux);
  __shared__ double smem[kEndsSmem];
  if (ui(gd->ends_tile))
    ends_tile_body<true>(ugeo(gd->lev[0].geo), ui(gd->ends_nseg), cp(gd->tab64_0), cp(gd->vol0), gp(rq->f),
                         gp((const double *)rq->u), nullptr, 0.0, nullptr, 0.0, gp(gd->us), gp(gd->r),
                         gp(gd->partial), ui(bg - ents[e].block0), smem);
  else
    begin_body(ugeo(gd->lev[0].geo), cp(gd->tab64_0), cp(gd->vol0), gp(rq->f), gp((const double *)rq->u),
               gp(gd->us), gp(gd->r), gp(gd->partial), ui(bg - ents[e].block0));
}

// One block per grid: the stopping rule into the state, then the initial
// norms and threshold (F_INIT).
__global__ __launch_bounds__(kBlock) void kb_init(const StageEnt *__restrict__ ents,
                                                  const ReqDev *__restrict__ reqs) {
  const GridDev *gd = gp(ents[blockIdx.x].g);
  const ReqDev *rq = gp(reqs + ents[blockIdx.x].aux);
  PcgState *st = gp(gd->st);
  if (threadIdx.x == 0) {
    st->maxiter = rq->maxiter;
    st->flexible = rq->flexible;
  }
  finalize_body(gp(gd->partial), ui(gd->nb_begin), 2, st, F_INIT, rq->rtol, rq->atol, rq->rel_to_rhs, 0, 1);
}

// End of the solves of a table: the deferred updates of the last iterations,
// u back in plane-major order and the partial sums of its true residual.
__global__ __launch_bounds__(kBlock) void kb_finish(const StageEnt *__restrict__ ents, int nent, int total,
                                                    const ReqDev *__restrict__ reqs) {
  const int bg = logical_block();
  if (bg >= total) return;
  const int e = find_ent(ents, nent, bg);
  const GridDev *gd = gp(ents[e].g);
  const ReqDev *rq = gp(reqs + ents[e].aux);
  const PcgState *st = gp(gd->st);
  const int K = ui(st->iter);
  const int with_p = ui(st->status) != -4 ? pending_at_end(K) : 0;
  const double alpha = with_p ? st->alpha : 0.0;
  const double alpha2 = with_p == 2 ? st->alpha_prev : 0.0;
  double *pk = gp(dir_dev(gd, K)), *pk1 = gp(dir_dev(gd, K - 1));
  __shared__ double smem[kEndsSmem];
  if (ui(gd->ends_tile)) {
    auto go = [&](auto wp) {
      ends_tile_body<false, decltype(wp)::value>(ugeo(gd->lev[0].geo), ui(gd->ends_nseg), cp(gd->tab64_0),
                                                 cp(gd->vol0), gp(rq->f), gp(gd->us), pk, alpha, pk1, alpha2,
                                                 gp(rq->u), nullptr, gp(gd->partial), ui(bg - ents[e].block0),
                                                 smem);
    };
    if (with_p == 2) go(std::integral_constant<int, 2>{});
    else if (with_p == 1) go(std::integral_constant<int, 1>{});
    else go(std::integral_constant<int, 0>{});
  } else
    finish_body(ugeo(gd->lev[0].geo), cp(gd->tab64_0), cp(gd->vol0), gp(rq->f), gp(gd->us), pk, alpha, pk1, alpha2,
                with_p, gp(rq->u), gp(gd->partial), ui(bg - ents[e].block0));
}

// one block per grid
__global__ __launch_bounds__(kBlock) void kb_finalize(const StageEnt *__restrict__ ents, int mode) {
  const GridDev *gd = gp(ents[blockIdx.x].g);
  const int nblk = ui(mode == F_ALPHA ? gd->nb_apply
                                      : (mode == F_TRUE ? gd->nb_finish
                                                        : (mode == F_BETA && gd->nb_dot ? gd->nb_dot
                                                                                        : (mode == F_CONV_PENDING ? gd->nb_upd
                                                                                                                  : gd->nb_flat))));
  const int nq = (mode == F_BETA || mode == F_TRUE) ? 2 : 1;
  finalize_body(gp(gd->partial), nblk, nq, gp(gd->st), mode, 0.0, 0.0, 0, 0, 1);
}

__global__ void kb_gather_states(const StageEnt *__restrict__ ents, int nent, PcgState *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nent) out[i] = *ents[i].g->st;
}

// ------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------
// Blocks of one grid in the grouped CG operator step.
int batch_apply_blocks(const ell_grid *g) {
  const Geo &G = g->lev[0].geo;
  return g->apply_tile ? (int)tile_blocks(G, g->apply_nseg) : stencil_blocks(2LL * G.H, 1);
}

// Blocks of the start and end kernels of one grid inside a grouped launch:
// the operator step's tiles times the k-segments, else 64 plane-major
// columns (start) or 64 split slots (end) per block.
int begin_blocks(const ell_grid *g) {
  const Geo &G = g->lev[0].geo;
  if (g->tiled_ends) return (int)tile_blocks(G, ends_nseg(g));
  return (int)(((long long)G.nx * G.ny + kSegCols - 1) / kSegCols);
}
int finish_blocks(const ell_grid *g) {
  if (g->tiled_ends) return (int)tile_blocks(g->lev[0].geo, ends_nseg(g));
  return (int)((2LL * g->lev[0].geo.H + kSegCols - 1) / kSegCols);
}

// The finest level's FP64 half-sweeps after the first take the tiled kernel
// (four or eight k-segments there); with at least two levels
// the last two post-smoothing half-sweeps also form the CG dots.
bool batch_tile(const ell_grid *g) {
  const int ns = g->lev[0].geo.nseg;
  return tile_ok(g, 0) && ((ns == 4 && seg_len(g->d.nz, 4) <= 32) || (ns == 8 && seg_len(g->d.nz, 8) <= 16));
}
bool batch_fused_dot(const ell_grid *g) { return batch_tile(g) && g->fused_dot && g->L >= 2 && g->d.nu_post >= 1; }
// The mixed-precision V-cycle's finest prolongation rides on the first FP64
// colour-1 post-smoothing sweep (bilinear, the tiled sweep; the colour-0
// sweep after it overwrites colour 0 of z without reading it).
bool batch_pro32(const ell_grid *g) {
  return g->prec != ELL_FP64 && g->fused_prolong && g->d.prolong == 0 && g->L >= 2 && g->d.nu_post >= 1 &&
         batch_tile(g);
}
// The residual update rides on the finest level's first pre-smoothing pair
// (four k-segments of at most 32 levels or eight of at most 16).
bool batch_fused_update(const ell_grid *g) {
  const Geo &G = g->lev[0].geo;
  const int Ls = seg_len(G.nz, G.nseg);
  return g->fused_update && g->L >= 2 && ((G.nseg == 8 && Ls <= 16) || (G.nseg == 4 && Ls <= 32));
}
// Blocks of the colour-c sweep of that pair for grid g (one slot each).
int batch_upd_blocks(const ell_grid *g, int c) {
  const Geo &G = g->lev[0].geo;
  if (c == 1 && g->prec == ELL_FP64 && batch_tile(g)) return smooth_tiles(G);
  return (int)(((c ? G.ncol1 : G.ncol0) + kSegCols - 1) / kSegCols);
}

int grid_dev_build(ell_grid *g) {
  if (g->L > kMaxLevels) return fail(ELL_ERR_INVALID, "too many levels for the batch engine");
  GridDev h;
  std::memset(&h, 0, sizeof(h));
  for (int l = 0; l < g->L; ++l) {
    h.lev[l].geo = g->lev[l].geo;
    h.lev[l].tab = g->lev[l].tab;
    h.lev[l].b = g->lev[l].b;
    h.lev[l].u = g->lev[l].u;
  }
  h.tab64_0 = g->tab64_0;
  h.vol0 = g->vol0;
  h.us = g->us;
  h.r = g->r;
  h.z = g->z;
  h.p = g->p;
  h.p2 = g->p2;
  h.p3 = g->p3;
  h.q = g->q;
  h.u32 = (float *)g->z32;
  h.partial = g->partial;
  h.st = g->st;
  h.n2 = g->n0 / 2;
  h.L = g->L;
  h.apply_tile = g->apply_tile;
  h.apply_nseg = g->apply_nseg;
  h.nb_apply = batch_apply_blocks(g);
  h.nb_flat = batch_flat_blocks(h.n2);
  h.prolong = g->d.prolong;
  h.nb_begin = begin_blocks(g);
  h.nb_finish = finish_blocks(g);
  h.ends_tile = g->tiled_ends;
  h.ends_nseg = ends_nseg(g);
  h.nb_tiles = batch_tile(g) ? smooth_tiles(g->lev[0].geo) : 0;
  h.nb_dot = batch_fused_dot(g) ? 2 * h.nb_tiles : 0;
  h.nb_upd0 = batch_fused_update(g) ? batch_upd_blocks(g, 0) : 0;
  h.nb_upd = batch_fused_update(g) ? h.nb_upd0 + batch_upd_blocks(g, 1) : 0;
  void *d = nullptr;
  CHK(dalloc(g, &d, sizeof(GridDev)));
  HIPCHK(hipMemcpy(d, &h, sizeof(GridDev), hipMemcpyHostToDevice));
  g->gdev = d;
  return ELL_OK;
}

bool batch_capable(const ell_grid *g, std::string *why) {
  const auto &d = g->d;
  if (d.rho != 1.0) { *why = "batched grids need rho = 1"; return false; }
  if (d.nu_pre < 1 || d.nu_post < 1 || d.nu_coarse < 1) { *why = "batched grids need nu >= 1"; return false; }
  // coarse levels may be one column wide: the segmented sweep then reads
  // zero-initialised, never-written entries for the missing faces and
  // multiplies them by zero coefficients
  if (!g->lev[0].geo.has_x || !g->lev[0].geo.has_y) {
    *why = "batched grids need nx, ny > 1 on the finest level";
    return false;
  }
  if (seg_len(g->d.nz, 4) > 64) { *why = "batched grids need nz <= 256"; return false; }
  if (g->prec != ELL_FP64 && !hybrid_ok(g)) { *why = "mixed precision batches need >= 2 levels"; return false; }
  return true;
}

struct Request {
  uint64_t ticket;
  ell_grid *g;
  const double *f;
  double *u;
  ell_solve_opts o;
  ell_solve_stats st;
  int rc = ELL_PENDING;
};

struct Ticket {
  std::vector<Request *> reqs;
  int remaining;
};

// One stage of a grouped iteration.
struct Stage {
  enum Kind { APPLY_DIR, UPDATE_R, DOTS, FINALIZE, SMOOTH, SMOOTH_TILE, SMOOTH_UPD, SMOOTH_TILE_UPD, RESTRICT,
              PROLONG, PROLONG_OUT, PROLONG_TILE, PROLONG_OUT_TILE, SMOOTH_TILE_PRO } kind;
  int level, colour, zero, role, mode;  // mode: finalize mode; SMOOTH_TILE: 1 with the fused dots
  int seg;                              // SMOOTH: register segment length (16/32/64)
  int nseg;                             // SMOOTH, SMOOTH_TILE(_PRO): k-segments (block of nseg wavefronts)
  int pair;                             // SMOOTH_TILE_PRO: paired loads of the coarse values
  size_t off;                           // offset of the entry table in the device buffer
  int nent, total;
};

}  // namespace ellb
using namespace ellb;

struct ell_batch {
  size_t budget = 0;
  size_t used = 0;
  hipStream_t stream = nullptr;
  std::vector<ell_grid *> grids;  // owned
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Request *> queue;
  std::map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  int poll_every = 4;
  // engine state (worker thread only)
  std::vector<Request *> active;
  std::vector<Stage> stages;
  StageEnt *d_ents = nullptr;
  StageEnt *h_ents = nullptr;  // pinned staging
  size_t ents_cap = 0;
  PcgState *d_states = nullptr;
  PcgState *h_states = nullptr;  // pinned
  int states_cap = 0;
  void *d_tx = nullptr;  // start / end tables (request records + entries)
  void *h_tx = nullptr;  // pinned staging
  size_t tx_cap = 0;
  // one grouped step captured as a graph (rebuilt with the stage tables)
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  bool dirty = true;
  int table_cycles = 0;  // cycles the current stage table has run
  int prec = -1;
  int nu_pre = -1, nu_post = -1;  // shared by every grid (one V-cycle schedule per step)
  std::string last_error;
  // statistics
  long long steps = 0;
};

namespace {

int batch_reserve(ell_batch *b, size_t ents, int states) {
  if (ents > b->ents_cap) {
    if (b->d_ents) (void)hipFree(b->d_ents);
    if (b->h_ents) (void)hipHostFree(b->h_ents);
    b->d_ents = nullptr;
    b->h_ents = nullptr;
    size_t cap = std::max<size_t>(ents, 2 * b->ents_cap);
    HIPCHK(hipMalloc((void **)&b->d_ents, cap * sizeof(StageEnt)));
    HIPCHK(hipHostMalloc((void **)&b->h_ents, cap * sizeof(StageEnt), hipHostMallocDefault));
    b->ents_cap = cap;
  }
  if (states > b->states_cap) {
    if (b->d_states) (void)hipFree(b->d_states);
    if (b->h_states) (void)hipHostFree(b->h_states);
    b->d_states = nullptr;
    b->h_states = nullptr;
    int cap = std::max(states, 2 * b->states_cap);
    HIPCHK(hipMalloc((void **)&b->d_states, cap * sizeof(PcgState)));
    HIPCHK(hipHostMalloc((void **)&b->h_states, cap * sizeof(PcgState), hipHostMallocDefault));
    b->states_cap = cap;
  }
  return ELL_OK;
}

int tx_reserve(ell_batch *b, size_t bytes) {
  if (bytes <= b->tx_cap) return ELL_OK;
  if (b->d_tx) (void)hipFree(b->d_tx);
  if (b->h_tx) (void)hipHostFree(b->h_tx);
  const size_t cap = std::max<size_t>(bytes, 2 * b->tx_cap);
  b->d_tx = nullptr;
  b->h_tx = nullptr;
  b->tx_cap = 0;
  HIPCHK(hipMalloc(&b->d_tx, cap));
  HIPCHK(hipHostMalloc(&b->h_tx, cap, hipHostMallocDefault));
  b->tx_cap = cap;
  return ELL_OK;
}

// Build the stage list and entry tables for the active grids.  The V-cycle of
// every grid follows its own depth: at depth d the grids with more levels
// pre-smooth and restrict, the grids whose coarsest level is d run their
// coarse sweeps (the first of them shares the pre-smoothing launches).
int batch_build(ell_batch *b) {
  std::vector<StageEnt> ents;
  b->stages.clear();
  const auto &A = b->active;
  const bool mixed = b->prec != ELL_FP64;
  auto add = [&](Stage st, const std::vector<ell_grid *> &gs, auto blocks_of) {
    if (gs.empty()) return;
    st.off = ents.size();
    int tot = 0;
    for (ell_grid *g : gs) {
      const int nb = blocks_of(g);
      if (nb <= 0) continue;  // e.g. the empty colour of a 1x1 level
      ents.push_back(StageEnt{(const GridDev *)g->gdev, tot, 0});
      tot += nb;
    }
    st.nent = (int)(ents.size() - st.off);
    if (st.nent == 0) return;
    st.total = tot;
    b->stages.push_back(st);
  };
  std::vector<ell_grid *> all;
  for (Request *r : A) all.push_back(r->g);
  auto one = [](ell_grid *) { return 1; };
  auto flat = [](ell_grid *g) { return batch_flat_blocks(g->n0 / 2); };
  auto apply = [](ell_grid *g) { return batch_apply_blocks(g); };
  auto cols = [](int l, int c) {
    return [l, c](ell_grid *g) {
      const Geo &G = g->lev[l].geo;
      return (int)(((c ? G.ncol1 : G.ncol0) + kSegCols - 1) / kSegCols);
    };
  };
  auto coarse_cols = [](int l) {
    return [l](ell_grid *g) { return (int)((2LL * g->lev[l + 1].geo.H + kSegCols - 1) / kSegCols); };
  };
  auto red_cols = [](int l) {
    return [l](ell_grid *g) { return (int)((g->lev[l].geo.ncol0 + kSegCols - 1) / kSegCols); };
  };
  auto seg_of = [](const std::vector<ell_grid *> &gs, int l) {
    int m = 16;
    for (ell_grid *g : gs) m = std::max(m, seg_len(g->lev[l].geo.nz, 4));
    return m <= 16 ? 16 : (m <= 32 ? 32 : 64);
  };
  // A half-sweep stage; the finest level's FP64 half-sweeps after the first
  // go to the tiled kernel for the grids that take it (last_post: the last
  // post-smoothing pair, with the fused CG dots where the grid has them).
  // The finest level's first pre-smoothing pair of the grids with the fused
  // residual update (head: the plain pair of a grid's first step; tail: the
  // pair with r -= alpha q at the end of every step, then the convergence
  // test); one stage per colour, k-segment count and kernel.
  auto add_upd_pair = [&](const std::vector<ell_grid *> &upd, bool head) {
    const int role = mixed ? ROLE_PRE32 : ROLE_FINE64;
    for (int c = 0; c < 2; ++c) {
      for (int ns : {4, 8}) {
        std::vector<ell_grid *> col, tile;
        for (ell_grid *g : upd) {
          if (g->lev[0].geo.nseg != ns) continue;
          (c == 1 && !mixed && batch_tile(g) ? tile : col).push_back(g);
        }
        Stage st{};
        st.level = 0;
        st.colour = c;
        st.zero = c == 0 ? 1 : 0;
        st.role = role;
        st.nseg = ns;
        st.mode = head ? 1 : 0;
        st.kind = Stage::SMOOTH_UPD;
        st.seg = ns == 8 ? 16 : seg_of(col, 0);
        add(st, col, [c](ell_grid *g) { return batch_upd_blocks(g, c); });
        st.kind = Stage::SMOOTH_TILE_UPD;
        st.seg = ns == 8 ? 16 : seg_of(tile, 0);
        add(st, tile, [c](ell_grid *g) { return batch_upd_blocks(g, c); });
      }
    }
    if (!head) {
      Stage fc{};
      fc.kind = Stage::FINALIZE;
      fc.mode = F_CONV_PENDING;
      add(fc, upd, one);
    }
  };
  // One stage per k-segment count: the finest level has four or eight.
  auto add_smooth = [&](const Stage &st, const std::vector<ell_grid *> &gs, bool last_post) {
    const int l = st.level;
    const bool tiled = st.role == ROLE_FINE64 && l == 0 && !st.zero;
    for (int ns : {4, 8}) {
      std::vector<ell_grid *> col, tile, tile_dot;
      for (ell_grid *g : gs) {
        if (g->lev[l].geo.nseg != ns) continue;
        if (!tiled || !batch_tile(g)) col.push_back(g);
        else if (last_post && batch_fused_dot(g)) tile_dot.push_back(g);
        else tile.push_back(g);
      }
      Stage cst = st;
      cst.nseg = ns;
      cst.seg = ns == 8 ? 16 : seg_of(col, l);
      add(cst, col, cols(l, st.colour));
      auto tiles = [](ell_grid *g) { return smooth_tiles(g->lev[0].geo); };
      Stage t = st;
      t.kind = Stage::SMOOTH_TILE;
      t.nseg = ns;
      t.mode = 0;
      t.seg = ns == 8 ? 16 : seg_of(tile, 0);
      add(t, tile, tiles);
      t.mode = 1;
      t.seg = ns == 8 ? 16 : seg_of(tile_dot, 0);
      add(t, tile_dot, tiles);
    }
  };
  // The fused colour-1 sweeps of the mixed-precision grids that take them
  // (the first post-smoothing sweep of the finest level).
  auto add_pro = [&](const std::vector<ell_grid *> &gs, bool last_post) {
    for (int ns : {4, 8}) {
      for (int pair = 1; pair >= 0; --pair) {
        std::vector<ell_grid *> plain, dot;
        for (ell_grid *g : gs) {
          if (g->lev[0].geo.nseg != ns || (int)pro32_pairs_ok(g->lev[1].geo, g->lev[1].u) != pair) continue;
          (last_post && batch_fused_dot(g) ? dot : plain).push_back(g);
        }
        auto tiles = [](ell_grid *g) { return smooth_tiles(g->lev[0].geo); };
        Stage t{};
        t.kind = Stage::SMOOTH_TILE_PRO;
        t.level = 0;
        t.colour = 1;
        t.role = ROLE_FINE64;
        t.nseg = ns;
        t.pair = pair;
        t.mode = 0;
        t.seg = ns == 8 ? 16 : seg_of(plain, 0);
        add(t, plain, tiles);
        t.mode = 1;
        t.seg = ns == 8 ? 16 : seg_of(dot, 0);
        add(t, dot, tiles);
      }
    }
  };
  // One step is iteration K of every active grid, in the order
  //   z = M r (V-cycle), <r,z> and <z,q>, beta (kappa at K = 1),
  //   p = z + beta p, q = A p and <p,q>, alpha, r -= alpha q, convergence;
  // the solution update of iteration K is deferred into step K + 1 (or the
  // end of the solve).  A grid admitted just before the step starts at K = 1.
  // For the grids with the fused residual update, r -= alpha q and the
  // convergence test ride on the first pre-smoothing pair of the next
  // V-cycle, run at the end of the step (the next step continues that
  // V-cycle); a grid's first step runs that pair, plain, at its start.
  Stage s0{};
  // V-cycle, down
  int Dmax = 0;
  for (ell_grid *g : all) Dmax = std::max(Dmax, g->L);
  const int nu_pre = all.empty() ? 1 : all[0]->d.nu_pre;
  const int nu_post = all.empty() ? 1 : all[0]->d.nu_post;
  for (int d = 0; d < Dmax; ++d) {
    std::vector<ell_grid *> deep, bottom, here;
    for (ell_grid *g : all) {
      if (d < g->L - 1) deep.push_back(g);
      else if (d == g->L - 1) bottom.push_back(g);
    }
    here = deep;
    here.insert(here.end(), bottom.begin(), bottom.end());
    if (here.empty()) continue;
    const int role = d == 0 ? (mixed ? ROLE_PRE32 : ROLE_FINE64) : ROLE_COARSE;
    int sweeps_shared = nu_pre;
    for (int it = 0; it < sweeps_shared; ++it) {
      // grids at their coarsest level take part in the first pair only if
      // they have at least one coarse sweep (nu_coarse >= 1, checked)
      std::vector<ell_grid *> gs = it == 0 ? here : deep;
      if (d == 0 && it == 0) {
        // the grids with the fused residual update run this pair here only in
        // their first step (the head form); later the end of the previous
        // step ran it
        std::vector<ell_grid *> upd, rest;
        for (ell_grid *g : gs) (batch_fused_update(g) ? upd : rest).push_back(g);
        add_upd_pair(upd, true);
        gs = rest;
      }
      for (int c = 0; c < 2; ++c) {
        Stage st{};
        st.kind = Stage::SMOOTH;
        st.level = d;
        st.colour = c;
        st.zero = (it == 0 && c == 0) ? 1 : 0;
        st.role = role;
        st.seg = seg_of(gs, d);
        add_smooth(st, gs, false);
      }
    }
    // remaining coarse sweeps of the grids whose coarsest level is d
    int maxc = 0;
    for (ell_grid *g : bottom) maxc = std::max(maxc, g->d.nu_coarse);
    for (int it = 1; it < maxc; ++it) {
      std::vector<ell_grid *> gs;
      for (ell_grid *g : bottom)
        if (g->d.nu_coarse > it) gs.push_back(g);
      for (int c = 0; c < 2; ++c) {
        Stage st{};
        st.kind = Stage::SMOOTH;
        st.level = d;
        st.colour = c;
        st.zero = 0;
        st.role = d == 0 ? (mixed ? ROLE_PRE32 : ROLE_FINE64) : ROLE_COARSE;
        st.seg = seg_of(gs, d);
        add_smooth(st, gs, false);
      }
    }
    if (!deep.empty()) {
      Stage st{};
      st.kind = Stage::RESTRICT;
      st.level = d;
      st.role = role;
      add(st, deep, coarse_cols(d));
    }
  }
  // V-cycle, up
  for (int d = Dmax - 2; d >= 0; --d) {
    std::vector<ell_grid *> gs;
    for (ell_grid *g : all)
      if (d < g->L - 1) gs.push_back(g);
    if (gs.empty()) continue;
    // mixed finest level: the grids whose prolongation rides on the first
    // colour-1 sweep take no prolongation stage
    std::vector<ell_grid *> pro, rest;
    for (ell_grid *g : gs) (d == 0 && mixed && batch_pro32(g) ? pro : rest).push_back(g);
    Stage st{};
    if (d == 0 && mixed) {
      st.kind = Stage::PROLONG_OUT;
      st.level = 0;
    } else {
      st.kind = Stage::PROLONG;
      st.level = d;
      st.role = d == 0 ? ROLE_FINE64 : ROLE_COARSE;
    }
    st.mode = gs[0]->d.prolong;
    {
      // bilinear prolongations on the tiled kernel where the level takes it
      std::vector<ell_grid *> col, tile;
      for (ell_grid *g : rest) {
        const Geo &F = g->lev[d].geo;
        (g->d.prolong == 0 && g->smooth_tile && F.has_x && F.ny % 2 == 0 ? tile : col).push_back(g);
      }
      add(st, col, red_cols(d));
      Stage t = st;
      t.kind = st.kind == Stage::PROLONG_OUT ? Stage::PROLONG_OUT_TILE : Stage::PROLONG_TILE;
      add(t, tile, [d](ell_grid *g) { return smooth_tiles(g->lev[d].geo); });
    }
    for (int it = 0; it < nu_post; ++it) {
      for (int c = 1; c >= 0; --c) {
        Stage sm{};
        sm.kind = Stage::SMOOTH;
        sm.level = d;
        sm.colour = c;
        sm.zero = 0;
        sm.role = d == 0 ? ROLE_FINE64 : ROLE_COARSE;
        sm.seg = seg_of(gs, d);
        if (it == 0 && c == 1 && !pro.empty()) {
          add_pro(pro, it == nu_post - 1);
          sm.seg = seg_of(rest, d);
          add_smooth(sm, rest, it == nu_post - 1);
        } else {
          add_smooth(sm, gs, it == nu_post - 1);
        }
      }
    }
  }
  std::vector<ell_grid *> nodot;  // grids without the fused dots
  for (ell_grid *g : all)
    if (!batch_fused_dot(g)) nodot.push_back(g);
  s0 = Stage{};
  s0.kind = Stage::DOTS;
  add(s0, nodot, flat);
  s0 = Stage{};
  s0.kind = Stage::FINALIZE;
  s0.mode = F_BETA;
  add(s0, all, one);
  // CG operator step, alpha, residual update, convergence
  s0 = Stage{};
  s0.kind = Stage::APPLY_DIR;
  add(s0, all, apply);
  s0 = Stage{};
  s0.kind = Stage::FINALIZE;
  s0.mode = F_ALPHA;
  add(s0, all, one);
  std::vector<ell_grid *> upd, noupd;  // grids with / without the fused residual update
  for (ell_grid *g : all) (batch_fused_update(g) ? upd : noupd).push_back(g);
  add_upd_pair(upd, false);
  s0 = Stage{};
  s0.kind = Stage::UPDATE_R;
  add(s0, noupd, flat);
  s0 = Stage{};
  s0.kind = Stage::FINALIZE;
  s0.mode = F_CONV;
  add(s0, noupd, one);
  // state gather table: one entry per active grid (reuses the FINALIZE layout)
  CHK(batch_reserve(b, ents.size() + 1, (int)all.size() + 1));
  if (!ents.empty()) {
    std::memcpy(b->h_ents, ents.data(), ents.size() * sizeof(StageEnt));
    HIPCHK(hipMemcpyAsync(b->d_ents, b->h_ents, ents.size() * sizeof(StageEnt), hipMemcpyHostToDevice,
                          b->stream));
  }
  b->dirty = false;
  return ELL_OK;
}

template <typename R, typename TB, bool FINE, int ROLE>
void launch_kb_smooth(const Stage &st, const StageEnt *e, int nb, hipStream_t s) {
  const int L = st.level, C = st.colour;
  if (st.nseg == 8) {  // the finest level with eight segments (at most 16 levels each)
    if (st.zero) kb_smooth<R, true, FINE, 16, TB, ROLE, 8><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total, L, C);
    else kb_smooth<R, false, FINE, 16, TB, ROLE, 8><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total, L, C);
    return;
  }
  if (st.zero) {
    if (st.seg == 16) kb_smooth<R, true, FINE, 16, TB, ROLE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, L, C);
    else if (st.seg == 32) kb_smooth<R, true, FINE, 32, TB, ROLE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, L, C);
    else kb_smooth<R, true, FINE, 64, TB, ROLE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, L, C);
  } else {
    if (st.seg == 16) kb_smooth<R, false, FINE, 16, TB, ROLE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, L, C);
    else if (st.seg == 32) kb_smooth<R, false, FINE, 32, TB, ROLE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, L, C);
    else kb_smooth<R, false, FINE, 64, TB, ROLE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, L, C);
  }
}

template <typename R, int ROLE, bool HEAD>
void launch_kb_smooth_upd(const Stage &st, const StageEnt *e, int nb, hipStream_t s) {
  const int C = st.colour;
  if (st.nseg == 8) {
    if (st.zero) kb_smooth_upd<R, true, 16, 8, ROLE, HEAD><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total, C);
    else kb_smooth_upd<R, false, 16, 8, ROLE, HEAD><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total, C);
  } else if (st.seg == 16) {
    if (st.zero) kb_smooth_upd<R, true, 16, 4, ROLE, HEAD><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, C);
    else kb_smooth_upd<R, false, 16, 4, ROLE, HEAD><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, C);
  } else {
    if (st.zero) kb_smooth_upd<R, true, 32, 4, ROLE, HEAD><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, C);
    else kb_smooth_upd<R, false, 32, 4, ROLE, HEAD><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, C);
  }
}

template <bool HEAD>
void launch_kb_tile_upd(const Stage &st, const StageEnt *e, int nb, hipStream_t s) {
  if (st.nseg == 8) kb_smooth_tile_upd<16, 8, HEAD><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total);
  else if (st.seg == 16) kb_smooth_tile_upd<16, 4, HEAD><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
  else kb_smooth_tile_upd<32, 4, HEAD><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
}

template <bool PAIR>
void launch_kb_pro32(const Stage &st, const StageEnt *e, int nb, hipStream_t s) {
  if (st.nseg == 8) {
    if (st.mode) kb_smooth_tile_pro32<16, 8, true, PAIR><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total);
    else kb_smooth_tile_pro32<16, 8, false, PAIR><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total);
  } else if (st.seg == 16) {
    if (st.mode) kb_smooth_tile_pro32<16, 4, true, PAIR><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
    else kb_smooth_tile_pro32<16, 4, false, PAIR><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
  } else {
    if (st.mode) kb_smooth_tile_pro32<32, 4, true, PAIR><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
    else kb_smooth_tile_pro32<32, 4, false, PAIR><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
  }
}

// Enqueue one grouped CG iteration for every active grid.
int batch_step(ell_batch *b) {
  hipStream_t s = b->stream;
  const bool mixed = b->prec != ELL_FP64;
  for (const Stage &st : b->stages) {
    const StageEnt *e = b->d_ents + st.off;
    const int nb = blocks8((long long)st.total * kBlock);
    switch (st.kind) {
      case Stage::APPLY_DIR: kb_apply_dir<<<nb, kBlock, 0, s>>>(e, st.nent, st.total); break;
      case Stage::UPDATE_R: kb_update_r<<<nb, kBlock, 0, s>>>(e, st.nent, st.total); break;
      case Stage::DOTS: kb_dots<<<nb, kBlock, 0, s>>>(e, st.nent, st.total); break;
      case Stage::SMOOTH_UPD:
        if (st.mode) {
          if (st.role == ROLE_PRE32) launch_kb_smooth_upd<float, ROLE_PRE32, true>(st, e, nb, s);
          else launch_kb_smooth_upd<double, ROLE_FINE64, true>(st, e, nb, s);
        } else {
          if (st.role == ROLE_PRE32) launch_kb_smooth_upd<float, ROLE_PRE32, false>(st, e, nb, s);
          else launch_kb_smooth_upd<double, ROLE_FINE64, false>(st, e, nb, s);
        }
        break;
      case Stage::SMOOTH_TILE_UPD:
        if (st.mode) launch_kb_tile_upd<true>(st, e, nb, s);
        else launch_kb_tile_upd<false>(st, e, nb, s);
        break;
      case Stage::SMOOTH_TILE:
        if (st.nseg == 8) {
          if (st.mode) kb_smooth_tile<16, 8, true><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total, st.colour);
          else kb_smooth_tile<16, 8, false><<<nb, 8 * 64, 0, s>>>(e, st.nent, st.total, st.colour);
        } else if (st.seg == 16) {
          if (st.mode) kb_smooth_tile<16, 4, true><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.colour);
          else kb_smooth_tile<16, 4, false><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.colour);
        } else {
          if (st.mode) kb_smooth_tile<32, 4, true><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.colour);
          else kb_smooth_tile<32, 4, false><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.colour);
        }
        break;
      case Stage::SMOOTH_TILE_PRO:
        if (st.pair) launch_kb_pro32<true>(st, e, nb, s);
        else launch_kb_pro32<false>(st, e, nb, s);
        break;
      case Stage::FINALIZE: kb_finalize<<<st.nent, kBlock, 0, s>>>(e, st.mode); break;
      case Stage::SMOOTH:
        if (st.role == ROLE_FINE64) launch_kb_smooth<double, double, true, ROLE_FINE64>(st, e, nb, s);
        else if (st.role == ROLE_PRE32) launch_kb_smooth<float, double, true, ROLE_PRE32>(st, e, nb, s);
        else if (mixed) launch_kb_smooth<float, float, false, ROLE_COARSE>(st, e, nb, s);
        else launch_kb_smooth<double, double, false, ROLE_COARSE>(st, e, nb, s);
        break;
      case Stage::RESTRICT:
        if (st.role == ROLE_FINE64) kb_restrict<double, double, ROLE_FINE64><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        else if (st.role == ROLE_PRE32) kb_restrict<float, double, ROLE_PRE32><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        else if (mixed) kb_restrict<float, float, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        else kb_restrict<double, double, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        break;
      case Stage::PROLONG:
        if (st.role == ROLE_FINE64) {
          if (st.mode == 1) kb_prolong<double, 1, ROLE_FINE64><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
          else kb_prolong<double, 0, ROLE_FINE64><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        } else if (mixed) {
          if (st.mode == 1) kb_prolong<float, 1, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
          else kb_prolong<float, 0, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        } else {
          if (st.mode == 1) kb_prolong<double, 1, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
          else kb_prolong<double, 0, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        }
        break;
      case Stage::PROLONG_TILE:
        if (st.role == ROLE_FINE64) kb_prolong_tile<double, ROLE_FINE64><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        else if (mixed) kb_prolong_tile<float, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        else kb_prolong_tile<double, ROLE_COARSE><<<nb, kBlock, 0, s>>>(e, st.nent, st.total, st.level);
        break;
      case Stage::PROLONG_OUT_TILE: kb_prolong_out_tile<<<nb, kBlock, 0, s>>>(e, st.nent, st.total); break;
      case Stage::PROLONG_OUT:
        if (st.mode == 1) kb_prolong_out<1><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
        else kb_prolong_out<0><<<nb, kBlock, 0, s>>>(e, st.nent, st.total);
        break;
    }
    CHK(check_launch("batched stage"));
  }
  return ELL_OK;
}

// Start (start = true: split-layout u and r, initial norms) or end (u back
// to the caller, true residual, final states into h_states in the order of
// rs, stream synchronised) of the solves of rs, grouped: one table upload
// and two launches for all of them.
int batch_edge(ell_batch *b, const std::vector<Request *> &rs, bool start) {
  hipStream_t s = b->stream;
  const int n = (int)rs.size();
  const size_t bytes = (size_t)n * sizeof(ReqDev) + 2 * (size_t)n * sizeof(StageEnt);
  CHK(tx_reserve(b, bytes));
  CHK(batch_reserve(b, 0, n + 1));
  ReqDev *hr = (ReqDev *)b->h_tx;
  StageEnt *he = (StageEnt *)(hr + n);
  StageEnt *h1 = he + n;
  int tot = 0;
  for (int i = 0; i < n; ++i) {
    const Request *r = rs[i];
    hr[i] = ReqDev{r->f, r->u, r->o.rtol, r->o.atol, r->o.rel_to_rhs, r->o.maxiter, r->o.flexible, 0};
    const GridDev *gd = (const GridDev *)r->g->gdev;
    he[i] = StageEnt{gd, tot, i};
    h1[i] = StageEnt{gd, i, i};
    tot += start ? begin_blocks(r->g) : finish_blocks(r->g);
  }
  HIPCHK(hipMemcpyAsync(b->d_tx, b->h_tx, bytes, hipMemcpyHostToDevice, s));
  const ReqDev *dr = (const ReqDev *)b->d_tx;
  const StageEnt *de = (const StageEnt *)(dr + n);
  const StageEnt *d1 = de + n;
  const int nb = blocks8((long long)tot * kBlock);
  if (start) {
    kb_begin<<<nb, kBlock, 0, s>>>(de, n, tot, dr);
    CHK(check_launch("kb_begin"));
    kb_init<<<n, kBlock, 0, s>>>(d1, dr);
    return check_launch("kb_init");
  }
  kb_finish<<<nb, kBlock, 0, s>>>(de, n, tot, dr);
  CHK(check_launch("kb_finish"));
  kb_finalize<<<n, kBlock, 0, s>>>(d1, F_TRUE);
  CHK(check_launch("kb_finalize"));
  kb_gather_states<<<(n + 63) / 64, 64, 0, s>>>(d1, n, b->d_states);
  CHK(check_launch("kb_gather_states"));
  HIPCHK(hipMemcpyAsync(b->h_states, b->d_states, n * sizeof(PcgState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return ELL_OK;
}

void drop_graph(ell_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
}

// Enqueue n grouped steps.  With graphs on, the step's launches are captured
// once per stage table (the tables, and with them every kernel argument, only
// change in batch_build) and the instantiated graph is launched n times; the
// step holds kernel launches only (no memset or copy nodes).  A table that
// runs a single step in its first cycle (a serving loop that polls every
// step, its set of solves changing from cycle to cycle) launches directly:
// the capture and instantiation would be host time the GPU waits for, spent
// on one launch; it is captured when it runs again.  A capture that fails
// switches the batch to direct launches.
int batch_steps(ell_batch *b, int n) {
  hipStream_t s = b->stream;
  if (b->use_graph && !b->gexec && (n > 1 || b->table_cycles > 0)) {
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      b->use_graph = false;
    } else {
      const int rc = batch_step(b);
      const hipError_t e = hipStreamEndCapture(s, &graph);
      if (rc != ELL_OK || e != hipSuccess || !graph ||
          hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        b->gexec = nullptr;
        b->use_graph = false;
      }
      if (graph) (void)hipGraphDestroy(graph);
    }
  }
  for (int k = 0; k < n; ++k) {
    if (b->gexec) {
      HIPCHK(hipGraphLaunch(b->gexec, s));
      b->steps++;
    } else {
      CHK(batch_step(b));
      b->steps++;
    }
  }
  b->table_cycles++;
  return ELL_OK;
}

void finish_ticket(ell_batch *b, Request *r) {
  std::lock_guard<std::mutex> lk(b->mu);
  auto it = b->tickets.find(r->ticket);
  if (it != b->tickets.end()) it->second.remaining--;
  r->g->busy = 0;
  b->cv_done.notify_all();
}

// Fail every request of rs with rc after draining the stream, so that no
// queued kernel still reads or writes their vectors once they are released.
void fail_all(ell_batch *b, std::vector<Request *> &rs, int rc) {
  (void)hipStreamSynchronize(b->stream);
  for (Request *r : rs) {
    r->rc = rc;
    finish_ticket(b, r);
  }
  rs.clear();
}

// One cycle: admit the queued requests whose grid is idle (their start runs
// grouped), poll_every grouped steps of every active grid, read the states
// back, end the finished solves (grouped) and hand back their tickets.
void worker_loop(ell_batch *b) {
  hipStream_t s = b->stream;
  for (;;) {
    std::vector<Request *> admit;
    {
      std::unique_lock<std::mutex> lk(b->mu);
      b->cv.wait(lk, [&] { return b->stop || !b->queue.empty() || !b->active.empty(); });
      if (b->stop && b->queue.empty() && b->active.empty()) return;
      // admit every queued request whose grid is idle (FIFO per grid)
      for (auto it = b->queue.begin(); it != b->queue.end();) {
        if (!(*it)->g->busy) {
          (*it)->g->busy = 1;
          admit.push_back(*it);
          it = b->queue.erase(it);
        } else {
          ++it;
        }
      }
    }
    int rc = ELL_OK;
    if (!admit.empty()) {
      if ((rc = batch_edge(b, admit, true)) != ELL_OK) {
        fail_all(b, admit, rc);
        fail_all(b, b->active, rc);
        b->dirty = true;
        continue;
      }
      b->active.insert(b->active.end(), admit.begin(), admit.end());
      b->dirty = true;
    }
    if (b->active.empty()) continue;
    if (b->dirty) {
      drop_graph(b);
      if ((rc = batch_build(b)) != ELL_OK) {
        fail_all(b, b->active, rc);
        continue;
      }
      b->table_cycles = 0;
    }
    rc = batch_steps(b, b->poll_every);
    // gather the states of the active grids with one copy
    const int n = (int)b->active.size();
    if (rc == ELL_OK) {
      const Stage *fin = nullptr;
      for (const Stage &st : b->stages)
        if (st.kind == Stage::FINALIZE) { fin = &st; break; }
      kb_gather_states<<<(n + 63) / 64, 64, 0, s>>>(b->d_ents + fin->off, n, b->d_states);
      rc = check_launch("kb_gather_states");
      if (rc == ELL_OK && hipMemcpyAsync(b->h_states, b->d_states, n * sizeof(PcgState), hipMemcpyDeviceToHost,
                                         s) != hipSuccess)
        rc = fail(ELL_ERR_HIP, "state copy failed");
      if (rc == ELL_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(ELL_ERR_HIP, "batch step failed");
    }
    if (rc != ELL_OK) {
      fail_all(b, b->active, rc);
      b->dirty = true;
      continue;
    }
    std::vector<Request *> ended, still;
    for (int i = 0; i < n; ++i) {
      Request *r = b->active[i];
      (b->h_states[i].done ? ended : still).push_back(r);
    }
    if (!ended.empty()) {
      rc = batch_edge(b, ended, false);
      for (size_t i = 0; i < ended.size(); ++i) {
        Request *r = ended[i];
        if (rc == ELL_OK) {
          *r->g->st_host = b->h_states[i];
          r->rc = stats_from_state(b->h_states[i], &r->st);
        } else {
          r->rc = rc;
        }
      }
      if (rc != ELL_OK) (void)hipStreamSynchronize(s);
      for (Request *r : ended) finish_ticket(b, r);
      b->dirty = true;
    }
    b->active.swap(still);
  }
}

}  // namespace

extern "C" {

int ell_batch_create(size_t hbm_budget_bytes, ell_batch **out) {
  if (!out) return fail(ELL_ERR_INVALID, "out is NULL");
  *out = nullptr;
  ell_batch *b = new ell_batch();
  b->budget = hbm_budget_bytes;
  b->use_graph = g_batch_graph != 0;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(ELL_ERR_HIP, "stream creation failed");
  }
  b->worker = std::thread(worker_loop, b);
  *out = b;
  return ELL_OK;
}

int ell_batch_grid(ell_batch *b, const ell_grid_desc *desc, ell_grid **out) {
  if (!b || !desc || !out) return fail(ELL_ERR_INVALID, "NULL argument");
  *out = nullptr;
  int L = 0;
  CHK(validate(desc, &L));
  const size_t need = grid_bytes(desc, L) + sizeof(GridDev);
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->used + need > b->budget)
      return fail(ELL_ERR_BUDGET, "grid needs %zu bytes, %zu of %zu in use", need, b->used, b->budget);
    if (b->prec != -1 && (b->prec == ELL_FP64) != (desc->precision == ELL_FP64))
      return fail(ELL_ERR_INVALID, "all grids of a batch use FP64 or all use the FP32 preconditioner");
    if (b->nu_pre != -1 && (b->nu_pre != desc->nu_pre || b->nu_post != desc->nu_post))
      return fail(ELL_ERR_INVALID, "all grids of a batch use the same pre- and post-smoothing counts");
  }
  ell_grid *g = nullptr;
  CHK(grid_create(desc, true, &g));
  std::string why;
  if (!batch_capable(g, &why)) {
    ell_grid_destroy(g);
    return fail(ELL_ERR_INVALID, "%s", why.c_str());
  }
  int rc = grid_dev_build(g);
  if (rc != ELL_OK) {
    ell_grid_destroy(g);
    return rc;
  }
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->used += need;
    b->grids.push_back(g);
    if (b->prec == -1) b->prec = desc->precision == ELL_FP64 ? ELL_FP64 : ELL_FP32_PRECOND;
    if (b->nu_pre == -1) {
      b->nu_pre = desc->nu_pre;
      b->nu_post = desc->nu_post;
    }
  }
  *out = g;
  return ELL_OK;
}

int ell_batch_release(ell_batch *b, ell_grid *g) {
  if (!b || !g) return fail(ELL_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(b->mu);
  auto it = std::find(b->grids.begin(), b->grids.end(), g);
  if (it == b->grids.end()) return fail(ELL_ERR_INVALID, "grid does not belong to this batch");
  if (g->busy) return fail(ELL_ERR_INVALID, "grid is in use");
  for (Request *r : b->queue)
    if (r->g == g) return fail(ELL_ERR_INVALID, "grid has queued requests");
  int L = g->L;
  b->used -= grid_bytes(&g->d, L) + sizeof(GridDev);
  b->grids.erase(it);
  ell_grid_destroy(g);
  return ELL_OK;
}

size_t ell_batch_bytes_in_use(const ell_batch *b) { return b ? b->used : 0; }

int ell_batch_submit(ell_batch *b, int32_t n, ell_grid *const *grids, const double *const *f, double *const *u,
                     const ell_solve_opts *opts, uint64_t *ticket_out) {
  if (!b || n <= 0 || !grids || !f || !u || !ticket_out) return fail(ELL_ERR_INVALID, "bad arguments");
  ell_solve_opts o;
  if (opts) o = *opts;
  else o = ell_solve_opts{1e-5, 0.0, 500, 1, 0, 4};
  if (o.maxiter <= 0 || !(o.rtol >= 0) || !(o.atol >= 0)) return fail(ELL_ERR_INVALID, "bad solve options");
  std::lock_guard<std::mutex> lk(b->mu);
  for (int i = 0; i < n; ++i) {
    if (std::find(b->grids.begin(), b->grids.end(), grids[i]) == b->grids.end())
      return fail(ELL_ERR_INVALID, "grid %d was not created by ell_batch_grid on this batch", i);
    if (!f[i] || !u[i]) return fail(ELL_ERR_INVALID, "NULL vector");
  }
  const uint64_t t = b->next_ticket++;
  Ticket tk;
  tk.remaining = n;
  for (int i = 0; i < n; ++i) {
    Request *r = new Request();
    r->ticket = t;
    r->g = grids[i];
    r->f = f[i];
    r->u = u[i];
    r->o = o;
    tk.reqs.push_back(r);
    b->queue.push_back(r);
  }
  if (o.poll_every > 0) b->poll_every = o.poll_every;
  b->tickets.emplace(t, std::move(tk));
  *ticket_out = t;
  b->cv.notify_all();
  return ELL_OK;
}

static int ticket_result(ell_batch *b, Ticket &tk, ell_solve_stats *stats) {
  int rc = ELL_OK;
  for (size_t i = 0; i < tk.reqs.size(); ++i) {
    Request *r = tk.reqs[i];
    if (stats) stats[i] = r->st;
    if (r->rc < 0 && (rc >= 0)) rc = r->rc;
    else if (r->rc == ELL_NOT_CONVERGED && rc == ELL_OK) rc = ELL_NOT_CONVERGED;
  }
  return rc;
}

int ell_batch_poll(ell_batch *b, uint64_t ticket, ell_solve_stats *stats) {
  if (!b) return fail(ELL_ERR_INVALID, "NULL batch");
  std::lock_guard<std::mutex> lk(b->mu);
  auto it = b->tickets.find(ticket);
  if (it == b->tickets.end()) return fail(ELL_ERR_INVALID, "unknown ticket");
  if (it->second.remaining > 0) return ELL_PENDING;
  return ticket_result(b, it->second, stats);
}

int ell_batch_wait(ell_batch *b, uint64_t ticket, ell_solve_stats *stats) {
  if (!b) return fail(ELL_ERR_INVALID, "NULL batch");
  std::unique_lock<std::mutex> lk(b->mu);
  auto it = b->tickets.find(ticket);
  if (it == b->tickets.end()) return fail(ELL_ERR_INVALID, "unknown ticket");
  b->cv_done.wait(lk, [&] { return it->second.remaining <= 0; });
  const int rc = ticket_result(b, it->second, stats);
  for (Request *r : it->second.reqs) delete r;
  b->tickets.erase(it);
  if (rc < 0) return fail(rc, "a solve of the batch failed");
  return rc;
}

int ell_batch_destroy(ell_batch *b) {
  if (!b) return ELL_OK;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->stop = true;
    b->cv.notify_all();
  }
  if (b->worker.joinable()) b->worker.join();
  for (auto &kv : b->tickets)
    for (Request *r : kv.second.reqs) delete r;
  for (ell_grid *g : b->grids) ell_grid_destroy(g);
  if (b->d_ents) (void)hipFree(b->d_ents);
  if (b->h_ents) (void)hipHostFree(b->h_ents);
  if (b->d_states) (void)hipFree(b->d_states);
  if (b->h_states) (void)hipHostFree(b->h_states);
  drop_graph(b);
  if (b->d_tx) (void)hipFree(b->d_tx);
  if (b->h_tx) (void)hipHostFree(b->h_tx);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return ELL_OK;
}

}  // extern "C"
