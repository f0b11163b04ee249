// Chebyshev recursion kernels: the forward step alpha_{m+1} = 2 H~ alpha_m -
// alpha_{m-1} with the probe moments mu_{m+1} = r^dag alpha_{m+1}, and the fused
// adjoint step that runs alpha backwards (reversible recursion), advances
// gamma_m = w C_{m+1} r + 2 H~ gamma_{m+1} - gamma_{m+2} and accumulates
// dOmega/dH~ on the stencil (App. B, eqs. alpha, dFdH, dalphadH, beta).
//
// Work decomposition (gfx950, wave64), sites tiled 8 x 4:
//  * Adjoint (both precisions) and FP64 forward: a wave owns one tile with TWO
//    lanes per site, one per Nambu row, so each lane keeps only its row's 18
//    coefficients of H~ (36 VGPRs in FP32) for the whole launch.  Lane l: site
//    s = l >> 1 of the tile (tx = s & 7, ty = s >> 3), row a = l & 1.
//  * FP32 forward (fwdp_body): two probes per wave step, one lane per (probe
//    slot, site) applying both Nambu rows, register coefficients of the
//    model's sparse rows, the tile's coefficient table staged once per block.
//  * The tile's input vector plus a one-site halo (10 x 6 = 60 records) is
//    staged through the wave's own LDS buffer, double-buffered: while one probe
//    (pair) is computed from LDS, the global loads of the next are in flight.
//  * The 4 waves of a block share the tile and take different probe subgroups
//    (PW probes each), so the adjoint's dOmega/dH~ contributions of 4 PW probes
//    are summed in LDS and written once per (site, probe range) per step.
//  * Blocks are dispatched round-robin over the 8 XCDs and scheduled so that
//    each XCD sweeps a spatially coherent part of the lattice (block_work):
//    the adjoint keeps one probe range per XCD on contiguous strips of tiles,
//    the forward sweeps one strip per XCD, range after range.
#include <hip/hip_ext.h>

#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "kpm_internal.h"

namespace kpm {

constexpr int TX = 8, TY = 4;                 // sites per wave tile
constexpr int HX = TX + 2, HY = TY + 2;       // halo tile
constexpr int HREC = HX * HY;                 // 60 staged records per vector
constexpr int WAVES = kBlock / 64;            // probe subgroups per block

template <typename V> using GPtr = const __attribute__((address_space(1))) V*;
template <typename V> using GPtrW = __attribute__((address_space(1))) V*;

// One site's record: (re, im) of Nambu components 0 and 1, loaded as one
// 16 B (FP32) or 32 B (FP64) vector.
typedef float F4 __attribute__((ext_vector_type(4)));
typedef double D4 __attribute__((ext_vector_type(4)));
template <typename V> struct RecT;
template <> struct RecT<float> { using T = F4; };
template <> struct RecT<double> { using T = D4; };

template <typename V>
__device__ __forceinline__ typename RecT<V>::T ldg_rec(const void* base, unsigned idx) {
  return ((GPtr<typename RecT<V>::T>)(base))[idx];
}
// one Nambu component of one site (record idx, component a)
template <typename V>
__device__ __forceinline__ Cx<V> ldg_comp(const void* base, unsigned idx, int a) {
  GPtr<V> p = ((GPtr<V>)(base)) + 4u * idx + 2u * a;
  return Cx<V>{p[0], p[1]};
}
template <typename V>
__device__ __forceinline__ void stg_comp(void* base, unsigned idx, int a, const Cx<V>& v) {
  GPtrW<V> p = ((GPtrW<V>)(base)) + 4u * idx + 2u * a;
  p[0] = v.x;
  p[1] = v.y;
}
template <typename V>
__device__ __forceinline__ Cx<V> comp_of(const typename RecT<V>::T& r, int b) {
  return b ? Cx<V>{r.z, r.w} : Cx<V>{r.x, r.y};
}

__device__ __forceinline__ long long ckpt_slot(int j, int k) { return 2LL * (j / k) + (j % k); }

// ------------------------------------------------------------- tile geometry
struct Lane {
  int s, a, tx, ty;      // tile site, Nambu row, tile coordinates
  int x, y;              // lattice coordinates (clamped into range)
  bool valid;            // site inside the lattice
  unsigned site;         // site index
  unsigned halo;         // record this lane stages (lanes < 60)
  int hoff[9];           // LDS record index of the 9 stencil neighbours
};

__device__ __forceinline__ Lane lane_geometry(const InstDev& I, int X0, int Y0, int lane) {
  Lane L;
  L.s = lane >> 1;
  L.a = lane & 1;
  L.tx = L.s & (TX - 1);
  L.ty = L.s / TX;
  int x = X0 + L.tx, y = Y0 + L.ty;
  L.valid = x < I.Lx && y < I.Ly;
  L.x = L.valid ? x : (x < I.Lx ? x : I.Lx - 1);
  L.y = L.valid ? y : (y < I.Ly ? y : I.Ly - 1);
  L.site = (unsigned)(L.y * I.Lx + L.x);
  // halo record h = lane: (hx, hy) in [0,10) x [0,6) -> lattice (X0 + hx - 1, Y0 + hy - 1) mod L
  const int h = lane < HREC ? lane : 0;
  // (a tile can be wider or taller than a small lattice: wrap by a full modulo)
  int hx = X0 + (h % HX) - 1, hy = Y0 + (h / HX) - 1;
  hx = ((hx % I.Lx) + I.Lx) % I.Lx;
  hy = ((hy % I.Ly) + I.Ly) % I.Ly;
  L.halo = (unsigned)(hy * I.Lx + hx);
  const int c = (L.ty + 1) * HX + (L.tx + 1);
  L.hoff[0] = c;
  L.hoff[1] = c + 1;            // +x
  L.hoff[2] = c + HX;           // +y
  L.hoff[3] = c + HX + 1;       // +x+y
  L.hoff[4] = c - HX + 1;       // +x-y
  L.hoff[5] = c - 1;            // -x
  L.hoff[6] = c - HX;           // -y
  L.hoff[7] = c - HX - 1;       // -x-y
  L.hoff[8] = c + HX - 1;       // -x+y
  return L;
}

// Row a of the site's 18 row coefficients of H~ (slot 2k + b, k = stencil slot).
template <typename V> struct RowCoef { Cx<V> c[18]; };

// 9 contiguous 64-lane loads from the lane-ordered coefficient table (the
// other waves of the block, on the same tile, find the lines in L1).
template <typename V>
__device__ __forceinline__ void load_row(RowCoef<V>& K, const InstDev& I, int tile, int lane) {
  using R4 = typename RecT<V>::T;
  GPtr<R4> base = (GPtr<R4>)(I.coef) + (size_t)tile * 9 * 64 + lane;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const R4 v = base[k * 64];
    K.c[2 * k] = Cx<V>{v.x, v.y};
    K.c[2 * k + 1] = Cx<V>{v.z, v.w};
  }
}

// ------------------------------------------------------------- probes
// Per-lane probe context: colour of the site in each group (used once per call
// by k_init, which evaluates the probes and writes the code table).
struct ProbeLane {
  int col[kMaxGroups];
};

__device__ __forceinline__ ProbeLane probe_lane(const InstDev& I, const Lane& L) {
  ProbeLane P;
#pragma unroll
  for (int g = 0; g < kMaxGroups; ++g) {
    P.col[g] = -1;
    if (g < I.ngroups && I.g[g].kind == kColoredZ4)
      P.col[g] = (L.x % I.g[g].px) + I.g[g].px * (L.y % I.g[g].py);
  }
  return P;
}

// Code k (entry = i^k) of probe p at the lane's (site, row); -1 for zero.
__device__ __forceinline__ int probe_code(const InstDev& I, const ProbeLane& P, const Lane& L,
                                          int p, double& w) {
  int k = -1;
  w = 0.0;
  for (int gi = 0; gi < I.ngroups; ++gi) {
    const GroupDev& g = I.g[gi];
    const int q = p - g.base;
    if (q < 0 || q >= g.nprobes) continue;
    w = g.weight;
    const unsigned I2 = 2u * L.site + (unsigned)L.a;
    if (g.kind == kUnit) {
      if ((unsigned)(g.first + q) == I2) k = 0;
    } else if (g.kind == kDenseZ4) {
      k = z4(g.seed, q, (int)I2);
    } else {
      const int per = g.px * g.py * (g.split ? 2 : 1);
      const int draw = q / per;
      int c = q - draw * per;
      int comp = -1;
      if (g.split) {
        comp = c & 1;
        c >>= 1;
      }
      if (P.col[gi] == c && (comp < 0 || comp == L.a)) k = z4(g.seed, draw, (int)I2);
    }
    break;
  }
  return k;
}

// Entry code of the lane's Nambu component from the probe's code byte.
__device__ __forceinline__ int lane_code(unsigned byte, int a) {
  const unsigned nib = (byte >> (4 * a)) & 0xFu;
  return (nib & 8u) ? (int)(nib & 3u) : -1;
}

__device__ __forceinline__ unsigned ldg_code(const InstDev& I, unsigned idx) {
  return ((GPtr<unsigned char>)(I.pcode))[idx];
}

// i^k s (0 for k < 0), without branches
template <typename V>
__device__ __forceinline__ Cx<V> phase_times(int k, V s) {
  const V sv = (k & 2) ? -s : s;
  const bool on = k >= 0;
  return Cx<V>{(on && !(k & 1)) ? sv : V(0), (on && (k & 1)) ? sv : V(0)};
}

// Re(conj(i^k) z) in FP64 (0 for k < 0).  Branches: for coloured and unit
// probes only one lane of a tile has k >= 0, and the others skip the work.
template <typename V>
__device__ __forceinline__ double re_conj_phase(int k, const Cx<V>& z) {
  double v = 0.0;
  if (k == 0) v = (double)z.x;
  else if (k == 1) v = (double)z.y;
  else if (k == 2) v = -(double)z.x;
  else if (k == 3) v = -(double)z.y;
  return v;
}

// 64-lane FP64 sum (every lane gets the total), fixed butterfly order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave sum of v over the lanes flagged nz: lanes read directly when at most
// two are set (coloured and unit probes: one site of a tile), else a butterfly.
// Wave-uniform result; deterministic for given data.
__device__ __forceinline__ double wave_moment(double v, bool nz) {
  unsigned long long mask = __ballot(nz);
  if (mask == 0ull) return 0.0;
  if (__popcll(mask) <= 2) {
    double s = read_lane(v, __ffsll((long long)mask) - 1);
    mask &= mask - 1ull;
    if (mask) s += read_lane(v, __ffsll((long long)mask) - 1);
    return s;
  }
  return wave_sum(nz ? v : 0.0);
}

// ------------------------------------------------------------- LDS staging
template <typename V> struct Stage {
  // [wave][buffer][vector][record]
  typename RecT<V>::T r[WAVES][2][2][HREC];
};


// Probe weight w_p, read through the constant address space: p is wave-uniform,
// so this is a scalar load, where a generic pointer would give a FLAT load that
// the compiler answers with full memory waits.  The table is written by an
// earlier kernel.
__device__ __forceinline__ double probe_weight(const InstDev& I, int p) {
  return ((const __attribute__((address_space(4))) double*)(I.pw))[p];
}

// Block -> (tile, probe range).  Blocks go to the 8 XCDs round-robin (XCD
// x = blockIdx % 8), and two schedules keep each XCD on a spatially coherent
// part of the lattice, so the halo rows neighbouring tiles share stay in its
// L2:
//  * RANGES (nranges divides 8): XCD x takes range x % nranges on the
//    (x / nranges)-th of 8 / nranges contiguous strips of `chunk` tiles; a
//    tile's coefficients and partial sums are touched by nranges XCDs.
//  * STRIPS: XCD x takes the x-th of 8 contiguous strips of `chunk` tiles and
//    sweeps it once per probe range, range after range; every tile's
//    coefficients are read by one XCD only, at the price of halo rows read
//    twice at the 8 strip boundaries.
//  * STRIP_TILES: XCD x takes the x-th of 8 contiguous strips and sweeps it
//    once, tile after tile, with all probe ranges of a tile in a row, so a
//    tile's coefficients are read from memory once and then from the XCD's L2.
//  Otherwise tile-major (range fastest).
//  * BALANCED (adjoint step of a single lattice): the (tile, probe) work is
//    cut into exactly as many equal contiguous shares as blocks fit on the
//    chip at once (adj_bal_body), so every CU gets the same work in one round.
enum : int { kSchedTileMajor = 0, kSchedRanges = 1, kSchedStrips = 2, kSchedStripTiles = 3,
             kSchedBalanced = 4 };
// tiles_x > 0: a single lattice, whose tile t sits at ((t % tiles_x) 8, (t / tiles_x) 4),
// so a block finds its tile without reading the tile table.
// BALANCED: nranges = probe groups, chunk = blocks in the grid, lg = probes per
// group, sl = partial-sum slices per group.
struct Sched { int nranges, chunk, ntiles, mode, tiles_x, lg, sl; };

__device__ __forceinline__ int4 tile_of(const Sched& sc, const int4* __restrict__ tmap, int tile) {
  if (sc.tiles_x > 0) return make_int4(0, (tile % sc.tiles_x) * TX, (tile / sc.tiles_x) * TY, tile);
  return tmap[tile];
}
__device__ __forceinline__ bool block_work(const Sched& sc, int& tile, int& range) {
  const int b = blockIdx.x;
  if (sc.mode == kSchedStrips) {
    const int x = b & 7, i = b >> 3;
    range = i / sc.chunk;
    tile = x * sc.chunk + (i - range * sc.chunk);
    return tile < sc.ntiles;
  }
  if (sc.mode == kSchedStripTiles) {
    const int x = b & 7, i = b >> 3;
    const int t = i / sc.nranges;
    range = i - t * sc.nranges;
    tile = x * sc.chunk + t;
    return tile < sc.ntiles;
  }
  if (sc.mode == kSchedRanges) {
    const int x = b & 7;
    range = x % sc.nranges;
    tile = (x / sc.nranges) * sc.chunk + (b >> 3);
    return tile < sc.ntiles;
  }
  tile = b / sc.nranges;
  range = b % sc.nranges;
  return true;
}

// wave index as a scalar (it is uniform across the wave)
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ------------------------------------------------------------- init
// Evaluates every probe once: alpha_0 = r (and its checkpoint), the code
// table pcode, the weight table pw and the mu_0 partials per tile.
template <typename V, int PW>
__global__ __launch_bounds__(kBlock) void k_init(const InstDev* __restrict__ insts,
                                                 const int4* __restrict__ tmap, Sched sc,
                                                 int k_ckpt, int store_ckpt) {
  int tile, range;
  if (!block_work(sc, tile, range)) return;               // block-uniform
  const int4 tm = tile_of(sc, tmap, tile);
  const InstDev& I = insts[tm.x];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int pbase = (range * WAVES + wave) * PW;
  if (pbase >= I.R) return;                              // wave-uniform, no barriers below
  const Lane L = lane_geometry(I, tm.y, tm.z, lane);
  const ProbeLane PL = probe_lane(I, L);
  const int pend = min(pbase + PW, I.R);
  for (int p = pbase; p < pend; ++p) {
    double w;
    const int k = probe_code(I, PL, L, p + I.poff, w);
    const Cx<V> r = phase_times<V>(k, V(1));
    const unsigned rec = (unsigned)(p * I.N) + L.site;
    const unsigned nib = k >= 0 ? (8u | (unsigned)k) : 0u;
    const unsigned other = (unsigned)__shfl_xor((int)nib, 1, 64);
    if (L.valid) {
      stg_comp<V>(I.A[0], rec, L.a, r);
      if (store_ckpt)
        stg_comp<V>((char*)I.ckpt + ckpt_slot(0, k_ckpt) * (long long)I.R * I.N * sizeof(typename RecT<V>::T),
                    rec, L.a, r);
      if (L.a == 0) I.pcode[rec] = (unsigned char)(nib | (other << 4));
    }
    if (tm.w == 0 && lane == 0) I.pw[p] = w;
    const double s = wave_moment(1.0, L.valid && k >= 0);
    if (lane == 0) I.mom[(long long)tm.w * I.R + p] = s;
  }
}

// ------------------------------------------------------------- addressing
// In the adjoint, probe vectors are addressed as a wave-uniform base (buffer +
// p N records, computed in scalar registers) plus a per-lane 32-bit byte
// offset fixed for the whole launch, so a load or store costs one 64-bit add
// per lane instead of an index multiply-add.
template <typename V> using C2 = V __attribute__((ext_vector_type(2)));

struct Off {
  unsigned halo;   // byte offset of the record this lane stages
  unsigned own;    // byte offset of the lane's own component (site, row a)
};

template <typename V>
__device__ __forceinline__ Off lane_offsets(const Lane& L) {
  constexpr unsigned RB = sizeof(typename RecT<V>::T), CB = RB / 2;
  return Off{L.halo * RB, L.site * RB + (unsigned)L.a * CB};
}

template <typename V>
__device__ __forceinline__ const char* probe_base(const void* buf, int p, int N) {
  return (const char*)buf + (size_t)p * (size_t)N * sizeof(typename RecT<V>::T);
}
template <typename V>
__device__ __forceinline__ typename RecT<V>::T ld_rec(const char* base, unsigned off) {
  return *(GPtr<typename RecT<V>::T>)(base + off);
}
template <typename V>
__device__ __forceinline__ Cx<V> ld_cx(const char* base, unsigned off) {
  const C2<V> v = *(GPtr<C2<V>>)(base + off);
  return Cx<V>{v.x, v.y};
}
template <typename V>
__device__ __forceinline__ void st_cx(const char* base, unsigned off, const Cx<V>& v) {
  C2<V> t;
  t.x = v.x;
  t.y = v.y;
  *(GPtrW<C2<V>>)(const_cast<char*>(base) + off) = t;
}
__device__ __forceinline__ unsigned ld_code(const InstDev& I, int p, const Lane& L) {
  return ((GPtr<unsigned char>)(I.pcode + (size_t)p * (size_t)I.N))[L.site];
}
// the lane's own Nambu component of a staged record (a half-record LDS read)
template <typename V>
__device__ __forceinline__ Cx<V> lds_own(const typename RecT<V>::T* rec, int a) {
  const C2<V> h = ((const C2<V>*)rec)[a];
  return Cx<V>{h.x, h.y};
}

// ------------------------------------------------------------- sparse rows
// In the model's Hamiltonian the on-site Nambu block and the next-nearest-
// neighbour blocks have no anomalous (pairing) entries: pairing lives on
// nearest-neighbour bonds only (App. A).  For records k = 0 (site), 3, 4
// (forward diagonal bonds) and 7, 8 (backward diagonal bonds) row a then only
// couples to component a.  In the adjoint step (two row products per probe) a
// wave whose lanes all see exact zeros there runs the 13-term rows instead of
// the 18-term ones; any other stencil keeps the full rows.  (The forward step
// keeps the full rows: measured on gfx950 the short rows did not pay there.)
__device__ __forceinline__ constexpr bool nambu_diag(int k) {
  return k == 0 || k == 3 || k == 4 || k == 7 || k == 8;
}

template <typename V>
__device__ __forceinline__ bool wave_sparse(const RowCoef<V>& K, int a) {
  bool z = true;
#pragma unroll
  for (int k = 0; k < 9; ++k)
    if (nambu_diag(k)) {
      const Cx<V> c = a ? K.c[2 * k] : K.c[2 * k + 1];
      z = z && c.x == V(0) && c.y == V(0);
    }
  return __all(z);
}

// Moves the coefficient (row a, component a) of those records to slot 2k.
template <typename V>
__device__ __forceinline__ void compact_row(RowCoef<V>& K, int a) {
#pragma unroll
  for (int k = 0; k < 9; ++k)
    if (nambu_diag(k)) K.c[2 * k] = a ? K.c[2 * k + 1] : K.c[2 * k];
}

// acc += row a of H~ times the staged vector (SP: compacted sparse row).
template <typename V, bool SP>
__device__ __forceinline__ void row_apply(Cx<V>& acc, const RowCoef<V>& K,
                                          const typename RecT<V>::T* lds, const Lane& L) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (SP && nambu_diag(k)) {
      cfma(acc, K.c[2 * k], lds_own<V>(lds + L.hoff[k], L.a));
    } else {
      const typename RecT<V>::T v = lds[L.hoff[k]];
      cfma(acc, K.c[2 * k + 0], comp_of<V>(v, 0));
      cfma(acc, K.c[2 * k + 1], comp_of<V>(v, 1));
    }
  }
}

// Address of a store that every lane issues: its own element, or the sink for
// lanes outside the lattice.  The empty asm hides the choice from the
// compiler, which would otherwise split the store into two conditional ones.
__device__ __forceinline__ const char* store_addr(bool valid, const char* own, const char* sink) {
  const char* a = valid ? own : sink;
  asm volatile("" : "+v"(a));
  return a;
}

// ------------------------------------------------------------- forward step
// The forward step keeps the loads of FPD probes in flight: a register ring of
// staged halo records, own-site values and code bytes.
constexpr int FPD = 2;

// alpha_{m+1} into A[(m+1)&1] (holding alpha_{m-1}) from alpha_m in A[m&1];
// m == 0: alpha_1 = H~ alpha_0.  Moment partial of alpha_{m+1} per (probe, tile).
// CK: this step's alpha_{m+1} is also a checkpoint.
// DBL (moment doubling, k_ckpt then carries M): instead of r^dag alpha_{m+1},
// the partials of alpha_{m+1}^dag alpha_{m+1} and Re(alpha_{m+1}^dag alpha_m)
// go to moment slots 2(m+1) and 2m+1 (when below M), from which
// mu_{2j} = 2 alpha_j^dag alpha_j - mu_0 and mu_{2j+1} = 2 Re(alpha_{j+1}^dag alpha_j) - mu_1.
// ACC (direct probing estimate, even m): also y += D_m alpha_m + D_{m+1}
// alpha_{m+1} for the lane's own component, y the FP64 records in G[0..1] and
// D in musum; ACC == 2 starts y (first pair).  y's own component rides in the
// same register ring as the other per-probe loads.
template <typename V, int PW, bool CK, bool DBL = false, int ACC = 0>
__device__ __forceinline__ void fwd_body(const InstDev* __restrict__ insts,
                                         const int4* __restrict__ tmap, Sched sc, int m,
                                         int k_ckpt) {
  using R4 = typename RecT<V>::T;
  __shared__ Stage<V> S;
  int tile, range;
  if (!block_work(sc, tile, range)) return;               // block-uniform
  const int4 tm = tile_of(sc, tmap, tile);
  const InstDev& I = insts[tm.x];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int pbase = (range * WAVES + wave) * PW;
  if (pbase >= I.R) return;                              // wave-uniform; waves never sync
  const int N = I.N;
  const Lane L = lane_geometry(I, tm.y, tm.z, lane);
  RowCoef<V> K;
  load_row<V>(K, I, tm.w, lane);
  const void* cur = I.A[m & 1];
  void* nxt = I.A[(m + 1) & 1];
  const int mo = m + 1;
  void* ckbuf = CK ? (void*)((char*)I.ckpt + ckpt_slot(mo, k_ckpt) * (long long)I.R * N * sizeof(R4))
                   : nullptr;
  // global (not generic) pointer: a generic store would be a FLAT access
  GPtrW<double> mom = (GPtrW<double>)(I.mom) + ((long long)mo * I.nchunk + tm.w) * I.R;
  const int Mtot = k_ckpt;                                  // DBL only
  GPtrW<double> momS = (GPtrW<double>)(I.mom) + ((long long)(2 * mo) * I.nchunk + tm.w) * I.R;
  GPtrW<double> momX = (GPtrW<double>)(I.mom) + ((long long)(2 * m + 1) * I.nchunk + tm.w) * I.R;
  double momx = 0.0;                                        // DBL: Re(alpha_{m+1}^dag alpha_m)
  const int pend = min(pbase + PW, I.R);
  // Every load and store of the probe loop is issued unconditionally (loads
  // past the wave's last probe re-read that probe; lanes outside the lattice
  // store to the sink), so the compiler's memory-wait counts are exact and a
  // wave waits for the loads it needs, not for its earlier stores.
  constexpr unsigned RB = sizeof(R4), CB = RB / 2;   // bytes of a record, of a component
  const char* sink_own = (const char*)I.sink + (unsigned)L.s * RB + (unsigned)L.a * CB;
  double momv = 0.0;                     // moment of probe pbase + lane, stored after the loop
  // ACC: y records (FP64, 32 B) and their sink slots; D_m, D_{m+1}
  const void* ybuf = I.G[0];
  const char* sink_y = (const char*)I.sink + (unsigned)L.s * 32u + (unsigned)L.a * 16u;
  const double Dm = ACC ? I.musum[m] : 0.0, Dm1 = ACC ? I.musum[m + 1] : 0.0;
  // Ring of FPD probes in flight.  A slot is refilled only after its values
  // have been consumed, so each load lands in the register it is read from
  // later (no copies, which would force an early wait for the load).
  R4 st[FPD];
  Cx<V> pq[FPD];
  unsigned cq[FPD];
  Cx<double> yq[FPD];
#pragma unroll
  for (int u = 0; u < FPD; ++u) {
    const int p = min(pbase + u, pend - 1);
    st[u] = ldg_rec<V>(cur, (unsigned)(p * N) + L.halo);
    pq[u] = ldg_comp<V>(nxt, (unsigned)(p * N) + L.site, L.a);
    cq[u] = ldg_code(I, (unsigned)(p * N) + L.site);
    if constexpr (ACC == 1) yq[u] = ldg_comp<double>(ybuf, (unsigned)(p * N) + L.site, L.a);
  }
  // Straight-line steps (a step past the wave's last probe recomputes the
  // last probe and stores to the sink), so that the wait counts are static.
  for (int p0 = pbase; p0 < pend; p0 += FPD) {
    double dsv[FPD], dxv[FPD];            // DBL: this lane's terms of the ring's probes
#pragma unroll
    for (int u = 0; u < FPD; ++u) {
      const int p = p0 + u;
      const bool live = L.valid && p < pend;
      R4* lds = S.r[wave][u & 1][0];
      if (lane < HREC) lds[lane] = st[u];
      __builtin_amdgcn_wave_barrier();
      const int pn = min(p + FPD, pend - 1);
      st[u] = ldg_rec<V>(cur, (unsigned)(pn * N) + L.halo);
      Cx<V> o{V(0), V(0)};
      row_apply<V, false>(o, K, lds, L);
      // m == 0: alpha_1 = H~ alpha_0 (prev is not read then: it may be any bits)
      const Cx<V> o2{fma(V(2), o.x, -pq[u].x), fma(V(2), o.y, -pq[u].y)};
      if (m > 0) o = o2;
      const int k = live ? lane_code(cq[u], L.a) : -1;
      pq[u] = ldg_comp<V>(nxt, (unsigned)(pn * N) + L.site, L.a);
      cq[u] = ldg_code(I, (unsigned)(pn * N) + L.site);
      const size_t own = (size_t)((unsigned)(p * N) + L.site) * RB + (unsigned)L.a * CB;
      st_cx<V>(store_addr(live, (const char*)nxt + own, sink_own), 0u, o);
      if (CK) st_cx<V>(store_addr(live, (const char*)ckbuf + own, sink_own), 0u, o);
      if constexpr (ACC != 0) {
        const Cx<V> am = lds_own<V>(lds + L.hoff[0], L.a);
        Cx<double> y = ACC == 1 ? yq[u] : Cx<double>{0.0, 0.0};
        y.x = fma(Dm, (double)am.x, y.x);
        y.y = fma(Dm, (double)am.y, y.y);
        y.x = fma(Dm1, (double)o.x, y.x);
        y.y = fma(Dm1, (double)o.y, y.y);
        if constexpr (ACC == 1) yq[u] = ldg_comp<double>(ybuf, (unsigned)(pn * N) + L.site, L.a);
        const size_t yown = (size_t)((unsigned)(p * N) + L.site) * 32u + (unsigned)L.a * 16u;
        st_cx<double>(store_addr(live, (const char*)ybuf + yown, sink_y), 0u, y);
      }
      if constexpr (DBL) {
        // own alpha_m component from the staged record; lanes outside the
        // lattice and repeated probes contribute nothing
        const Cx<V> am = lds_own<V>(lds + L.hoff[0], L.a);
        const double ox = (double)o.x, oy = (double)o.y;
        dsv[u] = live ? fma(ox, ox, oy * oy) : 0.0;
        dxv[u] = live ? fma(ox, (double)am.x, oy * (double)am.y) : 0.0;
      } else {
        const double v = wave_moment(re_conj_phase<V>(k, o), k >= 0);
        if (lane == p - pbase) momv = v;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if constexpr (DBL) {
      static_assert(FPD == 2, "the butterfly below reduces two probes' sums");
      // Transposed butterfly over the four sums (S, X of probes p0, p0 + 1):
      // the lane halves trade one probe's pair, the quarters one quantity,
      // then plain halving; quarter (u, q) ends with the sum of quantity q
      // (0: S, 1: X) of probe p0 + u.
      const bool hi = (lane & 32) != 0, q1 = (lane & 16) != 0;
      const double k0 = hi ? dsv[1] : dsv[0], k1 = hi ? dxv[1] : dxv[0];
      const double s0 = hi ? dsv[0] : dsv[1], s1 = hi ? dxv[0] : dxv[1];
      const double c0 = k0 + __shfl_xor(s0, 32, 64), c1 = k1 + __shfl_xor(s1, 32, 64);
      double d = (q1 ? c1 : c0) + __shfl_xor(q1 ? c0 : c1, 16, 64);
#pragma unroll
      for (int sh = 8; sh >= 1; sh >>= 1) d += __shfl_xor(d, sh, 64);
#pragma unroll
      for (int u = 0; u < FPD; ++u) {
        const double ssum = read_lane(d, 32 * u), xsum = read_lane(d, 32 * u + 16);
        if (lane == p0 + u - pbase) {
          momv = ssum;
          momx = xsum;
        }
      }
    }
  }
  if constexpr (DBL) {
    if (lane < pend - pbase) {
      if (2 * m + 1 < Mtot) momX[pbase + lane] = momx;
      if (2 * mo < Mtot) momS[pbase + lane] = momv;
    }
  } else {
    if (lane < pend - pbase) mom[pbase + lane] = momv;
  }
}

// ------------------------------------------------------------- forward step, FP32 pairs
// The FP32 forward step with two probes per wave step: each lane takes one
// probe slot q of the step and one tile site s (pair_geometry), and applies
// both Nambu rows of its site.  Per (site, probe) this halves the LDS reads (the 9 staged
// records serve both rows) and the global loads and stores (one 16 B record
// instead of two 8 B components), against one row per lane.
//
// Rows: in the model's h the on-site block is diagonal and real (pairing only
// on nearest-neighbour bonds, App. A), and the next-nearest-neighbour blocks
// are Nambu-diagonal.  Those 50 coefficients of the two rows stay in
// registers; the 20 others (the on-site (i0,i1) pair and the anomalous next-
// nearest-neighbour entries) are staged in LDS and used only by waves whose
// tile has one of them nonzero (a ballot at launch), so any stencil is exact.
// The factor 2 of the recursion is folded into the register coefficients and
// alpha_{m-1} seeds the accumulator: alpha_{m+1} = (2 H~) alpha_m - alpha_{m-1}
// (FIRST, m = 0: alpha_1 = (1/2)(2 H~) alpha_0).
//
// The probe loop is fully unrolled (PW/2 steps), so the ring of loads in
// flight (FPP steps ahead: both halo records, the own alpha_{m-1} record and
// the code byte) lives in fixed registers and every memory wait count is
// static; every load and store is issued on every path (clamped probe index,
// sink for lanes outside the lattice or past the wave's last probe).

// Staged halo of one probe: 6 rows of 10 records, rows PROW records apart,
// the two probe slots PREC records apart.  With these pitches the 128-bit
// reads of a wave (16-lane groups holding one tile row of both slots) hit
// distinct LDS banks; pitches of 10 / 72 cost about 4 conflict cycles per
// read (measured with SQ_LDS_BANK_CONFLICT on gfx950).
constexpr int PROW = 16;
constexpr int PREC = 104;    // >= 6 * PROW, and PREC = 8 (mod 16)
constexpr int FPP = 1;       // probe pairs in flight

struct PairLane {
  int s, q;
  bool valid;
  unsigned site, halo;
  int hw;                 // LDS record index this lane stages (halo lanes)
  int hoff[9];
};

// Lane l: tile row g = l >> 4, probe slot q = bit 3, column c = l & 7, so a
// group of 16 lanes reads one tile row of both slots: 8 consecutive staged
// records per slot.  Halo lane h (< 60) stages record (h % 10, h / 10) at
// row pitch PROW.
__device__ __forceinline__ PairLane pair_geometry(const InstDev& I, int X0, int Y0, int lane) {
  PairLane L;
  L.q = (lane >> 3) & 1;
  L.s = ((lane >> 4) << 3) | (lane & 7);
  const int tx = L.s & (TX - 1), ty = L.s / TX;
  const int x = X0 + tx, y = Y0 + ty;
  L.valid = x < I.Lx && y < I.Ly;
  const int xc = x < I.Lx ? x : I.Lx - 1, yc = y < I.Ly ? y : I.Ly - 1;
  L.site = (unsigned)(yc * I.Lx + xc);
  const int h = lane < HREC ? lane : 0;
  int hx = X0 + (h % HX) - 1, hy = Y0 + (h / HX) - 1;
  hx = ((hx % I.Lx) + I.Lx) % I.Lx;
  hy = ((hy % I.Ly) + I.Ly) % I.Ly;
  L.halo = (unsigned)(hy * I.Lx + hx);
  L.hw = (h / HX) * PROW + (h % HX);
  const int c = (ty + 1) * PROW + (tx + 1);
  L.hoff[0] = c;
  L.hoff[1] = c + 1;
  L.hoff[2] = c + PROW;
  L.hoff[3] = c + PROW + 1;
  L.hoff[4] = c - PROW + 1;
  L.hoff[5] = c - 1;
  L.hoff[6] = c - PROW;
  L.hoff[7] = c - PROW - 1;
  L.hoff[8] = c + PROW - 1;
  return L;
}

// Register coefficients of both rows of a site, scaled by 2 (records k:
// 0 site, 1 +x, 2 +y, 3 +x+y, 4 +x-y, 5 -x, 6 -y, 7 -x-y, 8 -x+y).
struct PairCoef {
  float d0, d1;             // 2 H~_{(i0),(i0)}, 2 H~_{(i1),(i1)} (real)
  Cx<float> nn[4][2][2];    // records 1, 2, 5, 6: [row][component]
  Cx<float> dg[4][2];       // records 3, 4, 7, 8: (row 0, comp 0), (row 1, comp 1)
};
__device__ __forceinline__ constexpr int nn_rec(int j) { return j < 2 ? 1 + j : 3 + j; }   // 1 2 5 6
__device__ __forceinline__ constexpr int dg_rec(int j) { return j < 2 ? 3 + j : 5 + j; }   // 3 4 7 8

// LDS of a forward block: the tile's lane-ordered coefficient table (read
// once per block, shared by its 4 waves) and each wave's double-buffered
// staging of the two probes' halo records.
struct PairStage {
  F4 coef[9][64];                   // [record][lane 2 s + row] (row, comp 0 | comp 1), unscaled
  F4 r[WAVES][2][2][PREC];          // [wave][buffer][slot][record]
};

__device__ __forceinline__ Cx<float> c2x(float re, float im, float f) { return Cx<float>{re * f, im * f}; }

// acc += c * (real r)
__device__ __forceinline__ void rfma(Cx<float>& acc, float c, float vx, float vy) {
  acc.x = fmaf(c, vx, acc.x);
  acc.y = fmaf(c, vy, acc.y);
}

// The coefficients outside the register set (FULL: the stencil has anomalous
// on-site or next-nearest-neighbour entries), read from the staged table:
// on-site (i0, i1) and (i1, i0), and per next-nearest record (row 0, comp 1)
// and (row 1, comp 0).  Scaled by 2 here.
template <bool FULL>
__device__ __forceinline__ void pair_rows(Cx<float>& o0, Cx<float>& o1, const PairCoef& K,
                                          const F4* lds, const PairLane& L, const F4 (*T)[64]) {
  const F4 v0 = lds[L.hoff[0]];
  rfma(o0, K.d0, v0.x, v0.y);
  rfma(o1, K.d1, v0.z, v0.w);
  if constexpr (FULL) {
    const F4 t0 = T[0][2 * L.s], t1 = T[0][2 * L.s + 1];
    cfma(o0, c2x(t0.z, t0.w, 2.f), Cx<float>{v0.z, v0.w});
    cfma(o1, c2x(t1.x, t1.y, 2.f), Cx<float>{v0.x, v0.y});
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const F4 v = lds[L.hoff[nn_rec(j)]];
    const Cx<float> a{v.x, v.y}, b{v.z, v.w};
    cfma(o0, K.nn[j][0][0], a);
    cfma(o0, K.nn[j][0][1], b);
    cfma(o1, K.nn[j][1][0], a);
    cfma(o1, K.nn[j][1][1], b);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const F4 v = lds[L.hoff[dg_rec(j)]];
    const Cx<float> a{v.x, v.y}, b{v.z, v.w};
    cfma(o0, K.dg[j][0], a);
    cfma(o1, K.dg[j][1], b);
    if constexpr (FULL) {
      const F4 t0 = T[dg_rec(j)][2 * L.s], t1 = T[dg_rec(j)][2 * L.s + 1];
      cfma(o0, c2x(t0.z, t0.w, 2.f), b);
      cfma(o1, c2x(t1.x, t1.y, 2.f), a);
    }
  }
}

// Re(conj(r_a) o_a) summed over the two Nambu components of a lane, from
// the probe's code byte (nibble a: 8 | k for the entry i^k, 0 for zero); FP64.
__device__ __forceinline__ double code_dot(unsigned cb, float x0, float y0, float x1, float y1) {
  const unsigned n0 = cb & 15u, n1 = (cb >> 4) & 15u;
  float v0 = (n0 & 1u) ? y0 : x0;
  v0 = (n0 & 2u) ? -v0 : v0;
  float v1 = (n1 & 1u) ? y1 : x1;
  v1 = (n1 & 2u) ? -v1 : v1;
  const double t0 = (n0 & 8u) ? (double)v0 : 0.0;
  const double t1 = (n1 & 8u) ? (double)v1 : 0.0;
  return t0 + t1;
}

// Sum of v over the lanes of each probe slot (slot q: lanes with bit 3 = q)
// flagged nz, in a fixed order: a slot with at most two such lanes reads them
// directly (coloured and unit probes), else a butterfly over the slot's 32
// lanes (lane distances 1, 2, 4, 16, 32).  s0, s1: the two slots' sums.
__device__ __forceinline__ void slot_moments(double v, bool nz, double& s0, double& s1) {
  const unsigned long long mask = __ballot(nz);
  const unsigned long long m0 = mask & 0x00FF00FF00FF00FFull, m1 = mask & 0xFF00FF00FF00FF00ull;
  double b0 = 0.0, b1 = 0.0;
  if (__popcll(m0) > 2 || __popcll(m1) > 2) {
    double t = nz ? v : 0.0;
    t += __shfl_xor(t, 1, 64);
    t += __shfl_xor(t, 2, 64);
    t += __shfl_xor(t, 4, 64);
    t += __shfl_xor(t, 16, 64);
    t += __shfl_xor(t, 32, 64);
    b0 = read_lane(t, 0);
    b1 = read_lane(t, 8);
  }
  auto direct = [&](unsigned long long m, double b) {
    if (__popcll(m) > 2) return b;
    double r = 0.0;
    if (m) {
      r = read_lane(v, __ffsll((long long)m) - 1);
      m &= m - 1ull;
      if (m) r += read_lane(v, __ffsll((long long)m) - 1);
    }
    return r;
  };
  s0 = direct(m0, b0);
  s1 = direct(m1, b1);
}

template <int PW, bool CK, bool FIRST>
__device__ __forceinline__ void fwdp_body(const InstDev* __restrict__ insts,
                                          const int4* __restrict__ tmap, Sched sc, int m,
                                          int k_ckpt) {
  static_assert(PW % 2 == 0, "two probes per wave step");
  constexpr int NP = PW / 2;
  __shared__ PairStage S;
  int tile, range;
  if (!block_work(sc, tile, range)) return;               // block-uniform
  const int4 tm = tile_of(sc, tmap, tile);
  const InstDev& I = insts[tm.x];
  if (range * WAVES * PW >= I.R) return;                 // block-uniform
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int pbase = (range * WAVES + wave) * PW;
  const bool has = pbase < I.R;                          // wave-uniform
  const int N = I.N;
  const PairLane L = pair_geometry(I, tm.y, tm.z, lane);
  const void* cur = I.A[m & 1];
  void* nxt = I.A[(m + 1) & 1];
  const int pend = has ? min(pbase + PW, I.R) : I.R;
  // ring of loads in flight; the first pair's loads are issued before the
  // block stages its coefficient table, so the two latencies overlap
  F4 h0[FPP], h1[FPP], pv[FPP];
  unsigned cd[FPP];
  auto issue_halo = [&](int j, int u) {
    const int p0 = min(pbase + 2 * j, pend - 1), p1 = min(pbase + 2 * j + 1, pend - 1);
    h0[u] = ldg_rec<float>(cur, (unsigned)(p0 * N) + L.halo);
    h1[u] = ldg_rec<float>(cur, (unsigned)(p1 * N) + L.halo);
  };
  auto issue_prev = [&](int j, int u) {
    const int p = min(pbase + 2 * j + L.q, pend - 1);
    if constexpr (!FIRST) pv[u] = ldg_rec<float>(nxt, (unsigned)(p * N) + L.site);
  };
  auto issue_code = [&](int j, int u) {
    const int p = min(pbase + 2 * j + L.q, pend - 1);
    cd[u] = ldg_code(I, (unsigned)(p * N) + L.site);
  };
  if (has) {
#pragma unroll
    for (int j = 0; j < FPP && j < NP; ++j) {
      issue_halo(j, j);
      issue_prev(j, j);
      issue_code(j, j);
    }
  }
  // the tile's coefficient table, staged once for the block's waves
  {
    GPtr<F4> src = (GPtr<F4>)(I.coef) + (size_t)tm.w * 9 * 64;
    for (int e = threadIdx.x; e < 9 * 64; e += kBlock) S.coef[e >> 6][e & 63] = src[e];
  }
  __syncthreads();
  if (!has) return;                                      // wave-uniform; no barrier below
  PairCoef K;
  bool extra_nz;
  {
    const F4 s0 = S.coef[0][2 * L.s], s1 = S.coef[0][2 * L.s + 1];
    K.d0 = 2.f * s0.x;
    K.d1 = 2.f * s1.z;
    bool nz = s0.z != 0.f || s0.w != 0.f || s1.x != 0.f || s1.y != 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const F4 r0 = S.coef[nn_rec(j)][2 * L.s], r1 = S.coef[nn_rec(j)][2 * L.s + 1];
      K.nn[j][0][0] = c2x(r0.x, r0.y, 2.f);
      K.nn[j][0][1] = c2x(r0.z, r0.w, 2.f);
      K.nn[j][1][0] = c2x(r1.x, r1.y, 2.f);
      K.nn[j][1][1] = c2x(r1.z, r1.w, 2.f);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const F4 r0 = S.coef[dg_rec(j)][2 * L.s], r1 = S.coef[dg_rec(j)][2 * L.s + 1];
      K.dg[j][0] = c2x(r0.x, r0.y, 2.f);
      K.dg[j][1] = c2x(r1.z, r1.w, 2.f);
      nz = nz || r0.z != 0.f || r0.w != 0.f || r1.x != 0.f || r1.y != 0.f;
    }
    extra_nz = __any(nz);
  }
  const int mo = m + 1;
  void* ckbuf = CK ? (void*)((char*)I.ckpt + ckpt_slot(mo, k_ckpt) * (long long)I.R * N * sizeof(F4))
                   : nullptr;
  GPtrW<double> mom = (GPtrW<double>)(I.mom) + ((long long)mo * I.nchunk + tm.w) * I.R;
  const char* sink = (const char*)I.sink + (unsigned)lane * 16u;
  double momv = 0.0;
  auto step = [&](auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int u = j % FPP;
      F4* buf = S.r[wave][j & 1][0];
      if (lane < HREC) {
        buf[L.hw] = h0[u];
        buf[PREC + L.hw] = h1[u];
      }
      __builtin_amdgcn_wave_barrier();
      if (j + FPP < NP) issue_halo(j + FPP, u);
      const int p = pbase + 2 * j + L.q;
      const bool live = L.valid && p < pend;
      Cx<float> o0{0.f, 0.f}, o1{0.f, 0.f};
      if constexpr (!FIRST) {
        o0 = Cx<float>{-pv[u].x, -pv[u].y};
        o1 = Cx<float>{-pv[u].z, -pv[u].w};
      }
      if (j + FPP < NP) issue_prev(j + FPP, u);
      pair_rows<FULL>(o0, o1, K, buf + L.q * PREC, L, S.coef);
      if constexpr (FIRST) {
        o0.x *= 0.5f; o0.y *= 0.5f; o1.x *= 0.5f; o1.y *= 0.5f;
      }
      const unsigned cb = live ? cd[u] : 0u;
      if (j + FPP < NP) issue_code(j + FPP, u);
      const size_t own = (size_t)((unsigned)(p < pend ? p : pend - 1) * (unsigned)N + L.site) * 16u;
      F4 ov;
      ov.x = o0.x; ov.y = o0.y; ov.z = o1.x; ov.w = o1.y;
      *(GPtrW<F4>)store_addr(live, (const char*)nxt + own, sink) = ov;
      if (CK) *(GPtrW<F4>)store_addr(live, (const char*)ckbuf + own, sink) = ov;
      const double t = code_dot(cb, o0.x, o0.y, o1.x, o1.y);
      double s0, s1;
      slot_moments(t, (cb & 0x88u) != 0u, s0, s1);
      if (lane == 2 * j) momv = s0;
      if (lane == 2 * j + 1) momv = s1;
      __builtin_amdgcn_wave_barrier();
    }
  };
  if (extra_nz) step(std::true_type{});
  else step(std::false_type{});
  if (lane < pend - pbase) mom[pbase + lane] = momv;
}

// ------------------------------------------------------------- adjoint
// gamma_{M-1} = 0, gamma_{M-2} = w C_{M-1} r; clears the dOmega/dH~ partials.
template <typename V, int PW>
__global__ __launch_bounds__(kBlock) void k_adj_init(const InstDev* __restrict__ insts,
                                                     const int4* __restrict__ tmap, Sched sc,
                                                     int M) {
  int tile, range;
  if (!block_work(sc, tile, range)) return;               // block-uniform
  const int4 tm = tile_of(sc, tmap, tile);
  const InstDev& I = insts[tm.x];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int pbase = (range * WAVES + wave) * PW;
  const Lane L = lane_geometry(I, tm.y, tm.z, lane);
  if (range * WAVES * PW >= I.R) return;
  // clear this (tile, range)'s partial sums: the two lanes of a site split the entries
  if (L.valid && wave == 0) {
    double2* gp = I.gpart + (long long)range * kNent * I.N;
    for (int e = L.a; e < kNent; e += 2) gp[(long long)e * I.N + L.site] = make_double2(0.0, 0.0);
  }
  if (pbase >= I.R) return;
  const double cM = I.C[M - 1];
  const int pend = min(pbase + PW, I.R);
  for (int p = pbase; p < pend; ++p) {
    const unsigned rec = (unsigned)(p * I.N) + L.site;
    if (L.valid) {
      const int k = lane_code(ldg_code(I, rec), L.a);
      stg_comp<V>(I.G[(M - 2) & 1], rec, L.a, phase_times<V>(k, (V)(I.pw[p] * cM)));
      stg_comp<V>(I.G[(M - 1) & 1], rec, L.a, Cx<V>{V(0), V(0)});
    }
  }
}

// One wave's probes of adjoint step m (see adj_body).  One probe is in
// flight: the halo records of the next probe are loaded right after this
// probe's are staged, its own-site values right after this probe's have been
// used, so every load lands in the register it is read from.  Every load and
// store is issued (clamped probe index; lanes outside the lattice store to the
// sink), so the wait counts are static and a wave waits for the loads it
// needs, not for its earlier stores.
template <typename V, bool SP, bool TAIL>
__device__ __forceinline__ void adj_loop(const InstDev& I, const Lane& L, const RowCoef<V>& K,
                                         typename RecT<V>::T (*stage)[2][HREC], int pbase,
                                         int pend, bool anchor, double Cm1, const void* Ax,
                                         const void* Gx, const void* Ay, const void* Gy,
                                         const void* Asrc, Cx<V> (&G)[10], int lane) {
  using R4 = typename RecT<V>::T;
  const int N = I.N;
  const Off O = lane_offsets<V>(L);
  const unsigned sown = (unsigned)lane * (unsigned)sizeof(Cx<V>);
  const char* sink = (const char*)I.sink;
  constexpr bool kEarlyOwn = sizeof(V) == 8;
  // a block's last waves can have no probe (pbase >= R): they load a valid
  // probe and skip the loop
  const int p0 = min(pbase, I.R - 1);
  R4 sa = ld_rec<V>(probe_base<V>(Ax, p0, N), O.halo);
  R4 sg = ld_rec<V>(probe_base<V>(Gx, p0, N), O.halo);
  Cx<V> aq{V(0), V(0)}, gq{V(0), V(0)};
  unsigned cq = 0u;
  if (!TAIL) {
    gq = ld_cx<V>(probe_base<V>(Gy, p0, N), O.own);
    aq = ld_cx<V>(probe_base<V>(Asrc, p0, N), O.own);
    cq = ld_code(I, p0, L);
  }
  int buf = 0;
  for (int p = pbase; p < pend; ++p, buf ^= 1) {
    const int pn = min(p + 1, pend - 1);
    R4* la = stage[buf][0];
    R4* lg = stage[buf][1];
    if (lane < HREC) {
      la[lane] = sa;
      lg[lane] = sg;
    }
    __builtin_amdgcn_wave_barrier();
    sa = ld_rec<V>(probe_base<V>(Ax, pn, N), O.halo);
    sg = ld_rec<V>(probe_base<V>(Gx, pn, N), O.halo);
    // FP64 (one wave per SIMD) issues the next own-site loads here, a step
    // earlier, into separate registers: its waves need the longer lead more
    // than they lose to the copies.
    Cx<V> gq_n{V(0), V(0)}, aq_n{V(0), V(0)};
    unsigned cq_n = 0u;
    if constexpr (kEarlyOwn) {
      if (!TAIL) {
        gq_n = ld_cx<V>(probe_base<V>(Gy, pn, N), O.own);
        aq_n = ld_cx<V>(probe_base<V>(Asrc, pn, N), O.own);
        cq_n = ld_code(I, pn, L);
      }
    }
    // dOmega/dH~ contribution of index src: conj(gamma_(i,a)) alpha_(j,b)
    const Cx<V> gi = lds_own<V>(lg + L.hoff[0], L.a);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const R4 v = la[L.hoff[1 + d]];
      cfma_conj(G[2 * d + 0], gi, comp_of<V>(v, 0));
      cfma_conj(G[2 * d + 1], gi, comp_of<V>(v, 1));
    }
    // a = 0: entries 16 (b = 0) and 18 (b = 1); a = 1: entry 17 (b = 1)
    cfma_conj(G[8], gi, lds_own<V>(la + L.hoff[0], L.a));
    cfma_conj(G[9], gi, lds_own<V>(la + L.hoff[0], 1));
    if (!TAIL) {
      // gamma_m row a
      Cx<V> gn{V(0), V(0)};
      row_apply<V, SP>(gn, K, lg, L);
      const Cx<V> sr = phase_times<V>(lane_code(cq, L.a), (V)(probe_weight(I, p) * Cm1));
      gn.x = fma(V(2), gn.x, sr.x - gq.x);
      gn.y = fma(V(2), gn.y, sr.y - gq.y);
      // alpha_m row a: checkpoint or reversed recursion
      Cx<V> an = aq;
      if (!anchor) {
        Cx<V> t{V(0), V(0)};
        row_apply<V, SP>(t, K, la, L);
        an.x = fma(V(2), t.x, -aq.x);
        an.y = fma(V(2), t.y, -aq.y);
      }
      if constexpr (kEarlyOwn) {
        gq = gq_n;
        aq = aq_n;
        cq = cq_n;
      } else {
        gq = ld_cx<V>(probe_base<V>(Gy, pn, N), O.own);
        aq = ld_cx<V>(probe_base<V>(Asrc, pn, N), O.own);
        cq = ld_code(I, pn, L);
      }
      st_cx<V>(store_addr(L.valid, probe_base<V>(Gy, p, N) + O.own, sink + sown), 0u, gn);
      st_cx<V>(store_addr(L.valid, probe_base<V>(Ay, p, N) + O.own, sink + sown + 2048u), 0u, an);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// LDS of an adjoint block: the waves' staged halos during the probe loop,
// then the per-wave partial sums (precision of V) for the block reduction.
template <typename V> union AdjShared {
  Stage<V> st;
  Cx<V> red[WAVES][kNent][TX * TY];
};

// Step m (0 <= m <= M-3): alpha_m, gamma_m from the m+1, m+2 vectors (the m+2
// buffers are overwritten), plus 2 conj(gamma_{m+1}) x alpha_{m+1} into the
// partial dOmega/dH~.  TAIL: only conj(gamma_0) x alpha_0 (weight 1).
// Lane (site, row a) accumulates the entries of row a: 4d + 2a + b (d < 4,
// b < 2) and the onsite ones (a = 0: 16, 18; a = 1: 17).
// One segment of a block's work: tile tm, this wave's probes [pbase, pend)
// (possibly none); the block's sums go to partial-sum slice `slice`.  Every
// wave of the block calls it (it synchronises the block).
template <typename V, bool TAIL>
__device__ __forceinline__ void adj_segment(const InstDev& I, const int4 tm, int pbase, int pend,
                                            int slice, int m, int k_ckpt, AdjShared<V>& S,
                                            int lane) {
  using R4 = typename RecT<V>::T;
  const int wave = wave_id();
  const int N = I.N;
  const Lane L = lane_geometry(I, tm.y, tm.z, lane);
  RowCoef<V> K;
  if (!TAIL) load_row<V>(K, I, tm.w, lane);
  const int src = TAIL ? m : m + 1;
  const void* Ax = I.A[src & 1];
  const void* Gx = I.G[src & 1];
  const void* Ay = I.A[m & 1];
  const void* Gy = I.G[m & 1];
  const double Cm1 = TAIL ? 0.0 : I.C[m + 1];
  const bool anchor = !TAIL && ((m % k_ckpt) <= 1);
  const void* ckbuf = anchor ? (const void*)((const char*)I.ckpt +
                                             ckpt_slot(m, k_ckpt) * (long long)I.R * N * sizeof(R4))
                             : nullptr;
  const void* Asrc = anchor ? ckbuf : Ay;
  Cx<V> G[10];
#pragma unroll
  for (int e = 0; e < 10; ++e) G[e] = Cx<V>{V(0), V(0)};
  // (FP64: full rows only; a second loop body would push the kernel past
  // 256 VGPRs into scratch)
  if constexpr (sizeof(V) == 4) {
    if (!TAIL && wave_sparse<V>(K, L.a)) {
      compact_row<V>(K, L.a);
      adj_loop<V, true, TAIL>(I, L, K, S.st.r[wave], pbase, pend, anchor, Cm1, Ax, Gx, Ay, Gy,
                              Asrc, G, lane);
    } else {
      adj_loop<V, false, TAIL>(I, L, K, S.st.r[wave], pbase, pend, anchor, Cm1, Ax, Gx, Ay, Gy,
                               Asrc, G, lane);
    }
  } else {
    adj_loop<V, false, TAIL>(I, L, K, S.st.r[wave], pbase, pend, anchor, Cm1, Ax, Gx, Ay, Gy,
                             Asrc, G, lane);
  }
  // sum the 4 waves' partials in LDS, then one read-modify-write per (site, entry)
  __syncthreads();
  const int s = L.s;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    S.red[wave][4 * d + 2 * L.a + 0][s] = G[2 * d];
    S.red[wave][4 * d + 2 * L.a + 1][s] = G[2 * d + 1];
  }
  if (L.a == 0) {
    S.red[wave][16][s] = G[8];
    S.red[wave][18][s] = G[9];
  } else {
    S.red[wave][17][s] = G[8];
  }
  __syncthreads();
  const double wgt = TAIL ? 1.0 : 2.0;
  double2* gp = I.gpart + (long long)slice * kNent * N;
  for (int q = threadIdx.x; q < kNent * TX * TY; q += kBlock) {
    const int e = q / (TX * TY), ss = q % (TX * TY);
    const int x = tm.y + (ss & (TX - 1)), y = tm.z + ss / TX;
    if (x >= I.Lx || y >= I.Ly) continue;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < WAVES; ++w2) {
      sx += (double)S.red[w2][e][ss].x;
      sy += (double)S.red[w2][e][ss].y;
    }
    const long long gi = (long long)e * N + y * I.Lx + x;
    double2 o = gp[gi];
    o.x += wgt * sx;
    o.y += wgt * sy;
    gp[gi] = o;
  }
}

// Block b = (tile, probe range) of the schedule; wave w runs the range's
// w-th PW probes; slice = range.
template <typename V, int PW, bool TAIL>
__device__ __forceinline__ void adj_body(const InstDev* __restrict__ insts,
                                         const int4* __restrict__ tmap, Sched sc, int m,
                                         int k_ckpt) {
  __shared__ AdjShared<V> S;
  int tile, range;
  if (!block_work(sc, tile, range)) return;               // block-uniform
  const int4 tm = tile_of(sc, tmap, tile);
  const InstDev& I = insts[tm.x];
  if (range * WAVES * PW >= I.R) return;                 // block-uniform
  const int pbase = (range * WAVES + wave_id()) * PW;
  adj_segment<V, TAIL>(I, tm, pbase, min(pbase + PW, I.R), range, m, k_ckpt, S, threadIdx.x & 63);
}

// Balanced schedule (single lattice).  The work units (probe group g, tile t,
// probe q of the group), ordered g, t, q, W = ntiles R of them, are cut into
// G = gridDim.x equal contiguous shares, G being the number of blocks that fit
// on the chip at once: every CU gets the same work in a single round.  Shares
// are dealt so that XCD x (blocks b = x mod 8) takes the x-th eighth of the
// order, a spatially coherent part of the lattice.  A share runs as segments
// (one per (g, t) it touches, at most a few), each split evenly over the
// block's waves.  The blocks touching one segment are consecutive in the
// order; the i-th of them adds into slice g sl + i, so no two blocks ever
// update the same partial sums in one launch (sl bounds that count; the host
// checks it and clears every slice before the first step).
template <typename V, bool TAIL>
__device__ __forceinline__ void adj_bal_body(const InstDev* __restrict__ insts,
                                             const int4* __restrict__ tmap, Sched sc, int m,
                                             int k_ckpt) {
  __shared__ AdjShared<V> S;
  const InstDev& I = insts[0];
  const int b = blockIdx.x;
  const long long G = sc.chunk, W = (long long)sc.ntiles * I.R;   // W < 2^31 (host check)
  const long long bl = (long long)(b & 7) * (G >> 3) + (b >> 3);
  // the share [u, u1) of the order, and its first segment's slice index: the
  // block's place among the blocks touching that segment (later segments
  // start inside the share, so the block is the first to touch them)
  int u = __builtin_amdgcn_readfirstlane((int)(bl * W / G));
  const int u1 = __builtin_amdgcn_readfirstlane((int)((bl + 1) * W / G));
  const int Lg = sc.lg;
  int sidx = __builtin_amdgcn_readfirstlane(
      (int)(bl - (((long long)(u / Lg) * Lg + 1) * G - 1) / W));
  const int wave = wave_id();
  while (u < u1) {                                       // block-uniform
    const int seg = u / Lg;
    const int q0 = u - seg * Lg;
    const int q1 = min(Lg, q0 + (u1 - u));
    const int g = seg / sc.ntiles, t = seg - g * sc.ntiles;
    const int lo = g * Lg + q0, n = q1 - q0;
    const int per = n >> 2, rem = n & 3;
    const int pbase = lo + wave * per + min(wave, rem);
    // the lane index is made opaque per segment, so that the compiler does not
    // hoist the lane's geometry out of this loop and hold it across the probe
    // loop (it would spill)
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    adj_segment<V, TAIL>(I, tile_of(sc, tmap, t), pbase, pbase + per + (wave < rem ? 1 : 0),
                         g * sc.sl + sidx, m, k_ckpt, S, lane);
    __syncthreads();                                     // LDS is staged again next segment
    u += n;
    sidx = 0;
  }
}

// Kernel entry points.  The FP32 kernels are held to 4 (forward) and 3
// (adjoint) waves per SIMD, i.e. at most 128 and 168 VGPRs, which leaves the
// register rings of loads in flight without spills.
template <typename V, int PW> struct StepKernels;
template <int PW> struct StepKernels<float, PW> {
  template <bool CK>
  static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
  void fwd(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
           int k_ckpt) {
    fwd_body<float, PW, CK>(insts, tmap, sc, m, k_ckpt);
  }
  template <bool CK, bool FIRST>
  static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
  void fwdp(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
            int k_ckpt) {
    if constexpr (PW % 2 == 0) fwdp_body<PW, CK, FIRST>(insts, tmap, sc, m, k_ckpt);
  }
  static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
  void fwd2(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
            int M) {
    fwd_body<float, PW, false, true>(insts, tmap, sc, m, M);
  }
  template <int ACC>
  static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
  void fwdacc(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
              int k_ckpt) {
    fwd_body<float, PW, false, false, ACC>(insts, tmap, sc, m, k_ckpt);
  }
  template <bool TAIL>
  static __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
  void adj(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
           int k_ckpt) {
    adj_body<float, PW, TAIL>(insts, tmap, sc, m, k_ckpt);
  }

};
template <int PW> struct StepKernels<double, PW> {
  template <bool CK>
  static __global__ __launch_bounds__(kBlock)
  void fwd(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
           int k_ckpt) {
    fwd_body<double, PW, CK>(insts, tmap, sc, m, k_ckpt);
  }
  static __global__ __launch_bounds__(kBlock)
  void fwd2(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
            int M) {
    fwd_body<double, PW, false, true>(insts, tmap, sc, m, M);
  }
  template <int ACC>
  static __global__ __launch_bounds__(kBlock)
  void fwdacc(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
              int k_ckpt) {
    fwd_body<double, PW, false, false, ACC>(insts, tmap, sc, m, k_ckpt);
  }
  template <bool TAIL>
  static __global__ __launch_bounds__(kBlock)
  void adj(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
           int k_ckpt) {
    adj_body<double, PW, TAIL>(insts, tmap, sc, m, k_ckpt);
  }
};

// Balanced-schedule adjoint steps (the probe block does not apply: a block's
// share sets its waves' probes).  Same register budgets as the adjoint above.
template <bool TAIL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
void k_adj_bal_f(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
                 int k_ckpt) {
  adj_bal_body<float, TAIL>(insts, tmap, sc, m, k_ckpt);
}
template <bool TAIL>
__global__ __launch_bounds__(kBlock)
void k_adj_bal_d(const InstDev* __restrict__ insts, const int4* __restrict__ tmap, Sched sc, int m,
                 int k_ckpt) {
  adj_bal_body<double, TAIL>(insts, tmap, sc, m, k_ckpt);
}

// p[0 .. n) = 0 (a fill kernel rather than a memset node, so graphs replay it)
__global__ __launch_bounds__(kBlock) void k_zero2(double2* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    p[i] = make_double2(0.0, 0.0);
}

// ------------------------------------------------------------- finishing
// mu[p][m] = sum over tiles (fixed order); also the [R][M] user copy.  Threads
// run over (m, p) with p fastest, so each pass of the tile loop reads
// consecutive probes' partials.
__global__ __launch_bounds__(kBlock) void k_mom_reduce(const InstDev* __restrict__ insts, int M,
                                                       double* __restrict__ mu_user) {
  const InstDev& I = insts[blockIdx.y];
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)I.R * M) return;
  const int m = (int)(t / I.R), p = (int)(t - (long long)m * I.R);
  const double* src = I.mom + (long long)m * I.nchunk * I.R + p;
  double s = 0.0;
  for (int c = 0; c < I.nchunk; ++c) s += src[(long long)c * I.R];
  I.musum[(long long)p * M + m] = s;
  if (mu_user) mu_user[(long long)p * M + m] = s;
}

// Moment doubling: slots m >= 2 of musum hold alpha_j^dag alpha_j (m = 2j) and
// Re(alpha_{j+1}^dag alpha_j) (m = 2j + 1); slots 0 and 1 are mu_0 and mu_1.
// mu_m = 2 musum_m - mu_{m & 1} (T_{2j} = 2 T_j^2 - 1, T_{2j+1} = 2 T_{j+1} T_j - T_1).
__global__ __launch_bounds__(kBlock) void k_mom_double(const InstDev* __restrict__ insts, int M,
                                                       double* __restrict__ mu_user) {
  const InstDev& I = insts[blockIdx.y];
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)I.R * M) return;
  const int p = (int)(t / M), m = (int)(t - (long long)p * M);
  double* row = I.musum + (long long)p * M;
  const double v = m >= 2 ? 2.0 * row[m] - row[m & 1] : row[m];
  if (m >= 2) row[m] = v;
  if (mu_user) mu_user[(long long)p * M + m] = v;
}

// Omega = sum_m C_m sum_p w_p mu_{p,m}: one block per (instance, 256 m),
// per-block partials in omega_part, summed in fixed order by k_omega_sum.
// Also the device check |mu_{p,m}| <= mu_{p,0} (|T_m(x)| <= 1 on [-1, 1]).
__global__ __launch_bounds__(kBlock) void k_omega(const InstDev* __restrict__ insts, int M) {
  const InstDev& I = insts[blockIdx.y];
  __shared__ double sh[kBlock];
  const int m = blockIdx.x * kBlock + threadIdx.x;
  double acc = 0.0;
  int bad = 0;
  if (m < M) {
    double s = 0.0;
    for (int gi = 0; gi < I.ngroups; ++gi) {
      const GroupDev& g = I.g[gi];
      double sg = 0.0;
      for (int q = 0; q < g.nprobes; ++q) {
        const int p = g.base + q;
        const double v = I.musum[(long long)p * M + m];
        const double v0 = I.musum[(long long)p * M];
        if (!isfinite(v) || fabs(v) > v0 * (1.0 + 1e-3) + 1e-9) bad = 1;
        sg += v;
      }
      s += g.weight * sg;
    }
    acc = I.C[m] * s;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (unsigned s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) I.opart[blockIdx.x] = sh[0];
  if (bad && I.status) *I.status = -4;
}

__global__ void k_omega_sum(const InstDev* __restrict__ insts, int nblk) {
  const InstDev& I = insts[blockIdx.x];
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += I.opart[b];
  if (I.omega) *I.omega = s;
}

// rho = omega_bar / a * sum over probe ranges of the partial dOmega/dH~.
__global__ __launch_bounds__(kBlock) void k_rho(const InstDev* __restrict__ insts,
                                                const int2* __restrict__ cmap) {
  const int2 cm = cmap[blockIdx.x];
  const InstDev& I = insts[cm.x];
  const int i = cm.y + threadIdx.x;
  if (i >= I.N) return;
  const double scale = (I.omega_bar ? *I.omega_bar : 1.0) / I.ab[0];
  const long long stride = (long long)kNent * I.N;
  bool bad = false;
  for (int e = 0; e < kNent; ++e) {
    double sx = 0.0, sy = 0.0;
    for (int b = 0; b < I.npb; ++b) {
      double2 v = I.gpart[b * stride + (long long)e * I.N + i];
      sx += v.x;
      sy += v.y;
    }
    if (e == 16 || e == 17) sy = 0.0;           // diagonal of a Hermitian matrix
    bad = bad || !isfinite(sx) || !isfinite(sy);
    I.rho[(long long)e * I.N + i] = make_double2(sx * scale, sy * scale);
  }
  if (bad && I.status) *I.status = -4;
}

// Order parameters from rho (kpm_density_matrix).
__global__ __launch_bounds__(kBlock) void k_map(int N, const double2* __restrict__ rho,
                                                double* n_up, double* n_dn, double2* chi_up,
                                                double2* chi_dn, double2* d_up, double2* d_dn) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  if (n_up) n_up[i] = rho[(long long)16 * N + i].x;
  if (n_dn) n_dn[i] = 1.0 - rho[(long long)17 * N + i].x;
  for (int d = 0; d < 4; ++d) {
    double2 r0 = rho[(long long)(4 * d + 0) * N + i], r1 = rho[(long long)(4 * d + 1) * N + i];
    double2 r2 = rho[(long long)(4 * d + 2) * N + i], r3 = rho[(long long)(4 * d + 3) * N + i];
    if (chi_up) chi_up[(long long)d * N + i] = r0;
    if (chi_dn) chi_dn[(long long)d * N + i] = make_double2(-r3.x, r3.y);
    if (d_up) d_up[(long long)d * N + i] = make_double2(-r1.x, r1.y);
    if (d_dn) d_dn[(long long)d * N + i] = make_double2(-r2.x, -r2.y);
  }
}

// ------------------------------------------------- direct probing estimate
// rho_IJ ~= (1/a) sum_p w_p conj(r_{p,I}) y_{p,J},  y_p = F_M'(H~) r_p
// = sum_m D_m alpha_{p,m} (the series of f' applied to each probe), which the
// forward steps with even m accumulate (fwd_body, ACC).  y is an FP64 record
// per (probe, site) in the adjoint buffers G[0..1], which the direct path
// does not use (2 FP32 records or 1 FP64 record of space each);
// D is kept in the first M doubles of musum, which the moment reduction
// overwrites only after the last accumulation.

// Coefficients of the derivative series: with e_M = e_{M+1} = 0,
// e_{k-1} = e_{k+1} + 2 k C_k (k = M-1 .. 1), D_0 = e_0 / 2, D_k = e_k.
// Unrolled, e_{k-1} = sum of T_j = 2 j C_j over j = k, k+2, ... <= M-1: a
// suffix sum within each parity of j.  One block per instance: thread t sums
// its contiguous chunk of j per parity, the chunks' totals are combined in
// LDS (each thread adds the totals above it, top down), and each thread then
// walks its chunk from the top, writing D.  Fixed order for given M.
__global__ __launch_bounds__(kBlock) void k_direct_coef(const InstDev* __restrict__ insts, int M) {
  __shared__ double tot[2][kBlock];
  const InstDev& I = insts[blockIdx.x];
  const double* __restrict__ C = I.C;
  double* __restrict__ D = I.musum;
  const int t = threadIdx.x;
  const int n = M - 1;                                  // j = 1 .. M-1
  const int chunk = (n + kBlock - 1) / kBlock;
  const int j0 = 1 + t * chunk, j1 = min(1 + (t + 1) * chunk, M);   // [j0, j1)
  double s[2] = {0.0, 0.0};
  for (int j = j1 - 1; j >= j0; --j) s[j & 1] += 2.0 * (double)j * C[j];
  tot[0][t] = s[0];
  tot[1][t] = s[1];
  __syncthreads();
  double acc[2] = {0.0, 0.0};
  for (int u = kBlock - 1; u > t; --u) {
    acc[0] += tot[0][u];
    acc[1] += tot[1][u];
  }
  for (int j = j1 - 1; j >= j0; --j) {
    acc[j & 1] += 2.0 * (double)j * C[j];
    D[j - 1] = j == 1 ? 0.5 * acc[1] : acc[j & 1];
  }
  if (t == 0) D[M - 1] = 0.0;
}

// One thread per site i: over the probes with a non-zero entry at (i, a),
// accumulate w conj(r_{(i,a)}) y_J for the stored entries of row (i, a):
// 4d + 2a + b (J = (i + d, b)), 16 / 18 (a = 0: J = (i, 0), (i, 1)), 17 (a = 1).
__global__ __launch_bounds__(kBlock) void k_rho_direct(const InstDev* __restrict__ insts,
                                                       const int2* __restrict__ cmap) {
  const int2 cm = cmap[blockIdx.x];
  const InstDev& I = insts[cm.x];
  const int i = cm.y + threadIdx.x;
  if (i >= I.N) return;
  const int Lx = I.Lx, Ly = I.Ly, N = I.N;
  const int x = i % Lx, y = i / Lx;
  int nb[4];
  {
    const int xp = (x + 1 == Lx) ? 0 : x + 1;
    const int yp = (y + 1 == Ly) ? 0 : y + 1, ym = (y == 0) ? Ly - 1 : y - 1;
    nb[0] = y * Lx + xp;
    nb[1] = yp * Lx + x;
    nb[2] = yp * Lx + xp;
    nb[3] = ym * Lx + xp;
  }
  Cx<double> acc[kNent];
#pragma unroll
  for (int e = 0; e < kNent; ++e) acc[e] = {0.0, 0.0};
  const unsigned char* code = I.pcode;
  for (int p = 0; p < I.R; ++p) {
    const unsigned byte = code[(size_t)p * N + i];
    if (byte == 0u) continue;
    const double w = I.pw[p];
    const long long base = (long long)p * N;
    const Rec<double> yi = ld_rec<double>(I.G[0], base + i);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const unsigned nib = (byte >> (4 * a)) & 15u;
      if (!(nib & 8u)) continue;
      // w conj(i^k)
      const Cx<double> r = phase_times<double>((int)(nib & 3u), w);
      const Cx<double> rc = {r.x, -r.y};
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const Rec<double> yj = ld_rec<double>(I.G[0], base + nb[d]);
        cfma(acc[4 * d + 2 * a + 0], rc, yj.c[0]);
        cfma(acc[4 * d + 2 * a + 1], rc, yj.c[1]);
      }
      if (a == 0) {
        cfma(acc[16], rc, yi.c[0]);
        cfma(acc[18], rc, yi.c[1]);
      } else {
        cfma(acc[17], rc, yi.c[1]);
      }
    }
  }
  const double scale = 1.0 / I.ab[0];
  bool bad = false;
  for (int e = 0; e < kNent; ++e) {
    double sx = acc[e].x * scale, sy = acc[e].y * scale;
    if (e == 16 || e == 17) sy = 0.0;
    bad = bad || !isfinite(sx) || !isfinite(sy);
    I.rho[(long long)e * N + i] = make_double2(sx, sy);
  }
  if (bad && I.status) *I.status = -4;
}

// ------------------------------------------------------------- profiling
// When enabled, runs of kWindow consecutive launches of the plain forward step
// (kind 1) or adjoint step (kind 3), one run starting every `every` launches of
// that kind, are timed by a pair of HIP events recorded by the dispatches
// themselves (hipExtLaunchKernelGGL): the start event by the run's first
// launch, the stop event by its last.  No marker packet sits between kernels,
// and the cost of the event signals is spread over the run.  A run is
// abandoned (its slot is not counted) when any other launch of this library
// comes before its last launch: another kernel, a step that is not the next
// one, another stream.  Kernels launched outside these launchers (moment
// reduction, copies) only follow a complete loop, whose runs have closed.
// The launches of a probe half on the second stream (the secondary stream of
// the launching thread) are neither timed nor counted as interruptions: a run
// on the caller's stream then covers steps whose other half runs beside it,
// so its launch average is the time per step of both halves.
namespace prof {
thread_local hipStream_t secondary = nullptr;
constexpr int kWindow = 16;
std::mutex mu;
bool on = false;
int every = kWindow;
int window = kWindow;
std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
std::vector<int> kind;      // 1 = forward step, 3 = adjoint step, 0 = abandoned
size_t used = 0;
// the open run: its slot, kind, stream, next expected step and launches left
struct Open {
  bool on = false;
  int kind = 0, next_m = 0, left = 0;
  hipStream_t s = nullptr;
  size_t slot = 0;
} open;

void abandon() {
  if (open.on) kind[open.slot] = 0;
  open.on = false;
}

// Events to attach to this launch (either may be null).  `k` is the launch's
// kind (1, 3, or 0 for any other launch), m its step, M the moment count.
void next(int k, int m, int M, hipStream_t s, hipEvent_t& a, hipEvent_t& b) {
  a = b = nullptr;
  if (secondary != nullptr && s == secondary) return;
  std::lock_guard<std::mutex> lk(mu);
  if (!on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    abandon();      // launches recorded into a graph are not timed
    return;
  }
  if (open.on) {
    if (k != open.kind || m != open.next_m || s != open.s) {
      abandon();
    } else {
      if (--open.left == 0) {
        b = pool[open.slot].second;
        open.on = false;
      } else {
        open.next_m += k == 1 ? 1 : -1;
      }
      return;
    }
  }
  // the forward loop runs m = 0 .. M-2 upwards, the adjoint m = M-3 .. 0 downwards
  const int pos = k == 1 ? m : M - 3 - m;
  const int last = k == 1 ? M - 2 : 0;
  if (k == 0 || pos % every != 0) return;
  if (k == 1 ? m + window - 1 > last : m - (window - 1) < last) return;
  if (used == pool.size()) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return;
    if (hipEventCreate(&e1) != hipSuccess) return;
    pool.emplace_back(e0, e1);
    kind.push_back(0);
  }
  a = pool[used].first;
  kind[used] = k;
  if (window == 1) {
    b = pool[used].second;
  } else {
    open.on = true;
    open.kind = k;
    open.s = s;
    open.slot = used;
    open.left = window - 1;
    open.next_m = k == 1 ? m + 1 : m - 1;
  }
  ++used;
}
}  // namespace prof

// The calling thread's second stream of probe halves (null: none).
void profile_secondary(hipStream_t s) { prof::secondary = s; }

hipError_t profile_begin(int every) {
  std::lock_guard<std::mutex> lk(prof::mu);
  prof::on = true;
  prof::every = every < 1 ? 1 : every;
  prof::window = std::min(prof::kWindow, prof::every);
  prof::used = 0;
  prof::open.on = false;
  return hipSuccess;
}

hipError_t profile_end(double* fwd_ms, int* nfwd, double* adj_ms, int* nadj) {
  std::lock_guard<std::mutex> lk(prof::mu);
  prof::on = false;
  prof::abandon();
  double f = 0.0, a = 0.0;
  int nf = 0, na = 0;
  for (size_t q = 0; q < prof::used; ++q) {
    if (prof::kind[q] == 0) continue;
    hipError_t e = hipEventSynchronize(prof::pool[q].second);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, prof::pool[q].first, prof::pool[q].second);
    if (e != hipSuccess) return e;
    if (prof::kind[q] == 1) {
      f += ms;
      nf += prof::window;
    } else {
      a += ms;
      na += prof::window;
    }
  }
  prof::used = 0;
  *fwd_ms = f;
  *nfwd = nf;
  *adj_ms = a;
  *nadj = na;
  return hipSuccess;
}

// ------------------------------------------------------------- launchers
// Schedule of a launch: the forward step (which 0, 1, 4, 5) sweeps strips
// (its coefficient table would otherwise be read by every XCD that holds a
// probe range), the adjoint (2, 3) keeps probe ranges per XCD.
// A requested schedule (0 tile-major, 1 ranges, 2 strips, 3 strips tile by
// tile) overrides the
// default; ranges needs a range count that divides 8, else tile-major runs.
static int sched_mode(int which, int nranges, int req) {
  int m = (which == 2 || which == 3) ? kSchedRanges : kSchedStrips;
  if (req >= kSchedTileMajor && req <= kSchedStripTiles) m = req;
  if (m == kSchedRanges && 8 % nranges != 0) return kSchedTileMajor;
  return m;
}

template <typename V, int PW>
static hipError_t launch_all(int sched, int which, const InstDev* insts, const int4* tmap,
                             int ntiles, int tiles_x, int nranges, int m, int M, int k_ckpt,
                             int flag, int4 bal, hipStream_t s) {
  if (which == 3 && sched == kSchedBalanced && bal.x > 0 && tiles_x > 0) {
    // balanced adjoint step: bal = (blocks, probes per group, slices per group, groups)
    const Sched sb{bal.w, bal.x, ntiles, kSchedBalanced, tiles_x, bal.y, bal.z};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    prof::next(flag == 0 ? 3 : 0, m, M, s, e0, e1);
    auto kern = sizeof(V) == 4 ? (flag ? k_adj_bal_f<true> : k_adj_bal_f<false>)
                               : (flag ? k_adj_bal_d<true> : k_adj_bal_d<false>);
    if (e0 != nullptr || e1 != nullptr)
      hipExtLaunchKernelGGL(kern, dim3(bal.x), dim3(kBlock), 0, s, e0, e1, 0, insts, tmap, sb, m, k_ckpt);
    else
      hipLaunchKernelGGL(kern, dim3(bal.x), dim3(kBlock), 0, s, insts, tmap, sb, m, k_ckpt);
    return hipGetLastError();
  }
  Sched sc{nranges, 0, ntiles, kSchedTileMajor, tiles_x, 0, 0};
  int nblocks = ntiles * nranges;
  const int mode = sched_mode(which, nranges, sched);
  if (mode == kSchedStrips || mode == kSchedStripTiles) {
    sc.mode = mode;
    sc.chunk = (ntiles + 7) / 8;
    nblocks = 8 * sc.chunk * nranges;
  } else if (mode == kSchedRanges && 8 % nranges == 0) {
    sc.mode = kSchedRanges;
    sc.chunk = (ntiles + 8 / nranges - 1) / (8 / nranges);
    nblocks = 8 * sc.chunk;
  }
  dim3 grid(nblocks), block(kBlock);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int pk = which == 1 ? 1 : (which == 3 && flag == 0) ? 3 : 0;
  prof::next(pk, m, M, s, e0, e1);
  const bool timed = e0 != nullptr || e1 != nullptr;
  switch (which) {
    case 0:
      hipLaunchKernelGGL((k_init<V, PW>), grid, block, 0, s, insts, tmap, sc, k_ckpt, flag);
      break;
    case 1: {
      // this step stores alpha_{m+1} as a checkpoint
      const bool ck = flag && ((m + 1) % k_ckpt) <= 1;
      auto kern = ck ? StepKernels<V, PW>::template fwd<true> : StepKernels<V, PW>::template fwd<false>;
      if constexpr (sizeof(V) == 4 && PW % 2 == 0) {
        // FP32: two probes per wave step
        if (m == 0)
          kern = ck ? StepKernels<V, PW>::template fwdp<true, true> : StepKernels<V, PW>::template fwdp<false, true>;
        else
          kern = ck ? StepKernels<V, PW>::template fwdp<true, false> : StepKernels<V, PW>::template fwdp<false, false>;
      }
      if (timed)
        hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, insts, tmap, sc, m, k_ckpt);
      else
        hipLaunchKernelGGL(kern, grid, block, 0, s, insts, tmap, sc, m, k_ckpt);
      break;
    }
    case 2:
      hipLaunchKernelGGL((k_adj_init<V, PW>), grid, block, 0, s, insts, tmap, sc, M);
      break;
    case 4:
      hipLaunchKernelGGL((StepKernels<V, PW>::fwd2), grid, block, 0, s, insts, tmap, sc, m, M);
      break;
    case 5: {
      // forward step with the direct-estimate accumulation (flag: first pair)
      auto kern = flag ? StepKernels<V, PW>::template fwdacc<2> : StepKernels<V, PW>::template fwdacc<1>;
      hipLaunchKernelGGL(kern, grid, block, 0, s, insts, tmap, sc, m, k_ckpt);
      break;
    }
    case 3: {
      auto kern = flag ? StepKernels<V, PW>::template adj<true> : StepKernels<V, PW>::template adj<false>;
      if (timed)
        hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, insts, tmap, sc, m, k_ckpt);
      else
        hipLaunchKernelGGL(kern, grid, block, 0, s, insts, tmap, sc, m, k_ckpt);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename V>
static hipError_t launch_p(int PW, int sched, int which, const InstDev* insts, const int4* tmap,
                           int ntiles, int tiles_x, int nranges, int m, int M, int k_ckpt, int flag,
                           int4 bal, hipStream_t s) {
  switch (PW) {
    case 1: return launch_all<V, 1>(sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt, flag, bal, s);
    case 2: return launch_all<V, 2>(sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt, flag, bal, s);
    case 4: return launch_all<V, 4>(sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt, flag, bal, s);
    case 8: return launch_all<V, 8>(sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt, flag, bal, s);
    case 16: return launch_all<V, 16>(sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt, flag, bal, s);
    case 32: return launch_all<V, 32>(sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt, flag, bal, s);
    default: return hipErrorInvalidValue;
  }
}

// tiles_x > 0 for a single lattice (tiles_x tiles per row), 0 for a batch (tile table)
hipError_t launch_cheb(bool fp32, int PW, int sched, int which, const InstDev* insts,
                       const int4* tmap, int ntiles, int tiles_x, int nranges, int m, int M,
                       int k_ckpt, int flag, int4 bal, hipStream_t s) {
  return fp32 ? launch_p<float>(PW, sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt,
                                flag, bal, s)
              : launch_p<double>(PW, sched, which, insts, tmap, ntiles, tiles_x, nranges, m, M, k_ckpt,
                                 flag, bal, s);
}

// Blocks of the balanced adjoint step that one CU holds at once.
hipError_t adj_bal_blocks_per_cu(bool fp32, int* nb) {
  *nb = 0;
  return fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_adj_bal_f<false>, kBlock, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_adj_bal_d<false>, kBlock, 0);
}

hipError_t launch_zero2(double2* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = std::min<long long>((n + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_zero2, dim3((unsigned)nb), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_mom_reduce(const InstDev* insts, int ninst, int maxRM, int M, double* mu_user,
                             hipStream_t s) {
  dim3 grid((maxRM + kBlock - 1) / kBlock, ninst);
  hipLaunchKernelGGL(k_mom_reduce, grid, dim3(kBlock), 0, s, insts, M, mu_user);
  return hipGetLastError();
}

hipError_t launch_omega(const InstDev* insts, int ninst, int M, hipStream_t s) {
  const int nblk = (M + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_omega, dim3(nblk, ninst), dim3(kBlock), 0, s, insts, M);
  hipLaunchKernelGGL(k_omega_sum, dim3(ninst), dim3(64), 0, s, insts, nblk);
  return hipGetLastError();
}

hipError_t launch_rho(const InstDev* insts, const int2* cmap, int nchunks, hipStream_t s) {
  hipLaunchKernelGGL(k_rho, dim3(nchunks), dim3(kBlock), 0, s, insts, cmap);
  return hipGetLastError();
}

hipError_t launch_mom_double(const InstDev* insts, int ninst, int maxRM, int M, double* mu_user,
                             hipStream_t s) {
  dim3 grid((maxRM + kBlock - 1) / kBlock, ninst);
  hipLaunchKernelGGL(k_mom_double, grid, dim3(kBlock), 0, s, insts, M, mu_user);
  return hipGetLastError();
}

hipError_t launch_direct_coef(const InstDev* insts, int ninst, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_direct_coef, dim3(ninst), dim3(kBlock), 0, s, insts, M);
  return hipGetLastError();
}

hipError_t launch_rho_direct(const InstDev* insts, const int2* cmap, int nchunks, hipStream_t s) {
  hipLaunchKernelGGL(k_rho_direct, dim3(nchunks), dim3(kBlock), 0, s, insts, cmap);
  return hipGetLastError();
}

hipError_t launch_map(int N, const double* rho, double* n_up, double* n_dn, double* chi_up,
                      double* chi_dn, double* d_up, double* d_dn, hipStream_t s) {
  hipLaunchKernelGGL(k_map, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N,
                     reinterpret_cast<const double2*>(rho), n_up, n_dn,
                     reinterpret_cast<double2*>(chi_up), reinterpret_cast<double2*>(chi_dn),
                     reinterpret_cast<double2*>(d_up), reinterpret_cast<double2*>(d_dn));
  return hipGetLastError();
}

}  // namespace kpm
