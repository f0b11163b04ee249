// Host side of the C ABI declared in include/kpm.h: argument validation,
// workspace layout, launch sequencing, batch plans (hipGraph) and the
// probes-per-thread autotuner.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include <sys/stat.h>

#include "../../include/kpm.h"
#include "kpm_internal.h"

namespace kpm {
hipError_t launch_build_h(const ModelDev&, const double*, const double*, const double*, double*,
                          hipStream_t);
hipError_t launch_build_vjp(const ModelDev&, const double*, const double*, const double*,
                            const double*, double*, double*, double*, hipStream_t);
hipError_t launch_build_sdw(const ModelDev&, const double*, const double*, const double*,
                            const double*, const double*, const double*, double*, hipStream_t);
hipError_t launch_build_sdw_vjp(const ModelDev&, const double*, const double*, const double*,
                                const double*, const double*, const double*, const double*, double*,
                                double*, double*, double*, double*, double*, hipStream_t);
hipError_t launch_bounds(int, int, const double*, double*, hipStream_t);
hipError_t launch_rescale(const InstDev*, const int4*, int, bool, hipStream_t);
hipError_t launch_coeffs(int, int, double, const double*, double*, hipStream_t);
hipError_t launch_cheb(bool, int, int, int, const InstDev*, const int4*, int, int, int, int, int, int,
                       int, int4, hipStream_t);
hipError_t adj_bal_blocks_per_cu(bool, int*);
hipError_t launch_zero2(double2*, long long, hipStream_t);
hipError_t launch_mom_reduce(const InstDev*, int, int, int, double*, hipStream_t);
hipError_t launch_omega(const InstDev*, int, int, hipStream_t);
hipError_t launch_rho(const InstDev*, const int2*, int, hipStream_t);
hipError_t launch_map(int, const double*, double*, double*, double*, double*, double*, double*,
                      hipStream_t);
hipError_t launch_direct_coef(const InstDev*, int, int, hipStream_t);
hipError_t launch_mom_double(const InstDev*, int, int, int, double*, hipStream_t);
hipError_t launch_ldos(const InstDev*, int, int, const double*, int, double*, hipStream_t);
hipError_t launch_rho_direct(const InstDev*, const int2*, int, hipStream_t);
hipError_t profile_begin(int);
hipError_t profile_end(double*, int*, double*, int*);
void profile_secondary(hipStream_t);

// Sets every instance's status word (a kernel, not a memset, so that the
// sequence can be captured in a hipGraph).
__global__ void k_set_status(const InstDev* __restrict__ insts, int ninst, int v) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ninst && insts[k].status) *insts[k].status = v;
}
}  // namespace kpm

using namespace kpm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxN = 1 << 26;
constexpr int kMaxR = 1 << 20;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

#define KPM_HIP(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return KPM_EDEVICE; \
  } while (0)

bool valid_lattice(const kpm_lattice* L) {
  if (!L) return false;
  if (L->Lx < 3 || L->Ly < 3) return false;
  if ((L->n_vortex % 2) != 0) return false;
  long long N = (long long)L->Lx * L->Ly;
  return N <= kMaxN;
}

long long group_nprobes(const kpm_probe_group& g) {
  if (g.kind == KPM_PROBE_COLORED_Z4)
    return (long long)g.count * g.px * g.py * (g.split_nambu ? 2 : 1);
  return g.count;
}

// Probe-vector records are addressed with 32-bit record indices p * N + site,
// and one Nambu component's element offset (4 values per record) must fit in
// 32 bits as well.
bool records_fit(const kpm_lattice* L, int R) {
  return (long long)R * L->Lx * L->Ly < (1LL << 30);
}

// Fills the device group table; returns R or < 0.
int build_groups(const kpm_lattice* L, const kpm_probes* pr, GroupDev* out, int* ng) {
  if (!pr || !pr->groups || pr->ngroups < 1 || pr->ngroups > KPM_MAX_PROBE_GROUPS) return -1;
  const long long N = (long long)L->Lx * L->Ly;
  long long R = 0;
  for (int k = 0; k < pr->ngroups; ++k) {
    const kpm_probe_group& g = pr->groups[k];
    if (g.count < 1 || !std::isfinite(g.weight)) return -1;
    switch (g.kind) {
      case KPM_PROBE_UNIT:
        if (g.first < 0 || (long long)g.first + g.count > 2 * N) return -1;
        break;
      case KPM_PROBE_DENSE_Z4:
        break;
      case KPM_PROBE_COLORED_Z4:
        if (g.px < 1 || g.py < 1 || g.px > L->Lx || g.py > L->Ly) return -1;
        if (g.split_nambu != 0 && g.split_nambu != 1) return -1;
        break;
      default:
        return -1;
    }
    const long long np = group_nprobes(g);
    if (np < 1 || np > kMaxR) return -1;
    if (out) {
      GroupDev& d = out[k];
      d.kind = g.kind;
      d.count = g.count;
      d.px = g.px;
      d.py = g.py;
      d.split = g.split_nambu;
      d.first = g.first;
      d.nprobes = (int)np;
      d.base = (int)R;
      d.seed = g.seed;
      d.weight = g.weight;
    }
    R += np;
    if (R > kMaxR) return -1;
  }
  if (ng) *ng = pr->ngroups;
  return (int)R;
}

bool valid_P(int P) { return P == 1 || P == 2 || P == 4 || P == 8 || P == 16 || P == 32; }

constexpr int kTX = 8, kTY = 4, kWaves = kBlock / 64;   // recursion tile and waves per block

// Probes per wave (P), from the measured behaviour of the 100x100 workload:
// the forward step wants many short waves (the largest P <= 8 that still gives
// ~8 waves per SIMD of the 256 CUs in one launch), the adjoint step wants few
// probe ranges (each range adds a read-modify-write of the FP64 partial sums and
// a pass over the coefficient table) as long as every SIMD still gets ~2 waves,
// and a range count that divides 8 or is a multiple of 8, so that every XCD
// keeps to its own probe ranges (block_work).
int waves_for(long long tiles_total, int Rmax, int P) {
  return (int)std::min<long long>(tiles_total * ((Rmax + kWaves * P - 1) / (kWaves * P)) * kWaves,
                                  1LL << 30);
}

int auto_probe_fwd(long long tiles_total, int Rmax) {
  int P = 8;
  while (P > 1 && waves_for(tiles_total, Rmax, P) < 256 * 4 * 8) P /= 2;
  return P;
}

int auto_probe_adj(long long tiles_total, int Rmax) {
  for (int P = 32; P > 1; P /= 2) {
    const int nr = (Rmax + kWaves * P - 1) / (kWaves * P);
    if ((8 % nr == 0 || nr % 8 == 0) && waves_for(tiles_total, Rmax, P) >= 256 * 4 * 2) return P;
  }
  return 1;
}

std::mutex g_mu;
int g_probe_block = 0;   // 0 = automatic
int g_sched_f = KPM_SCHED_DEFAULT, g_sched_a = KPM_SCHED_DEFAULT;   // single-lattice schedules

// Partial-sum slices of an instance's buffer: ceil(R / 4) ranges of P = 1,
// plus one for probe halves.
int gpart_slices(int R) { return (R + kWaves - 1) / kWaves + 1; }

// ------------------------------------------------------------ instance layout
struct Sizes {
  int N, R, M, nchunk, ntile;
  size_t rec, coef, vec, gvec, ckpt, mom, musum, gpart, pcode, pw, sink;
  long long nslots;
};

// fwd_only: the forward recursion and moments alone (no gamma vectors,
// checkpoints or adjoint partial sums).
Sizes sizes(const kpm_lattice* L, int R, int M, int k, bool fp32, bool fwd_only = false) {
  Sizes z{};
  z.N = L->Lx * L->Ly;
  z.R = R;
  z.M = M;
  z.nchunk = (z.N + kBlock - 1) / kBlock;
  z.ntile = ((L->Lx + kTX - 1) / kTX) * ((L->Ly + kTY - 1) / kTY);
  z.rec = fp32 ? 16 : 32;
  z.coef = align_up((size_t)z.ntile * 9 * 64 * 4 * (fp32 ? 4 : 8));
  z.vec = align_up((size_t)R * z.N * z.rec);
  z.nslots = 2LL * ((M - 1) / k + 1);
  z.ckpt = align_up((size_t)R * z.N * z.rec * (size_t)z.nslots);
  z.mom = align_up(sizeof(double) * (size_t)M * R * z.ntile);
  z.musum = align_up(sizeof(double) * (size_t)M * R);
  // one [19][N] FP64 slice per adjoint probe range; a range holds kWaves * P
  // probes, so P = 1 (the smallest block) needs the most ranges, and probe
  // halves one more (their ranges round up separately)
  z.gpart = align_up(sizeof(double) * 2 * kNent * (size_t)z.N * (size_t)gpart_slices(R));
  z.pcode = align_up((size_t)R * z.N);
  z.pw = align_up(sizeof(double) * (size_t)R);
  z.sink = align_up(4096);
  z.gvec = z.vec;
  if (fwd_only) z.gvec = z.ckpt = z.gpart = 0;
  return z;
}

size_t inst_bytes(const Sizes& z) {
  return align_up(sizeof(int)) + z.coef + 2 * z.vec + 2 * z.gvec + z.ckpt + z.mom + z.musum + z.gpart +
         align_up(sizeof(double) * ((z.M + kBlock - 1) / kBlock)) + z.pcode + z.pw + z.sink;
}

// Carve one instance's buffers out of `base` (which must hold inst_bytes).
void carve(InstDev& I, const Sizes& z, char* base) {
  char* o = base;
  I.status = reinterpret_cast<int*>(o);   o += align_up(sizeof(int));
  I.coef = o;                             o += z.coef;
  I.A[0] = o;                             o += z.vec;
  I.A[1] = o;                             o += z.vec;
  I.G[0] = o;                             o += z.gvec;
  I.G[1] = o;                             o += z.gvec;
  I.ckpt = o;                             o += z.ckpt;
  I.mom = reinterpret_cast<double*>(o);   o += z.mom;
  I.musum = reinterpret_cast<double*>(o); o += z.musum;
  I.gpart = reinterpret_cast<double2*>(o); o += z.gpart;
  I.opart = reinterpret_cast<double*>(o);  o += align_up(sizeof(double) * ((z.M + kBlock - 1) / kBlock));
  I.pcode = reinterpret_cast<unsigned char*>(o); o += z.pcode;
  I.pw = reinterpret_cast<double*>(o);
  o += z.pw;
  I.sink = o;
}

// ------------------------------------------------------------ run context
struct Ctx {
  std::vector<InstDev> inst;
  std::vector<int2> cmap;     // 256-site chunks (element-wise kernels)
  std::vector<int4> tmap;     // (instance, X0, Y0, tile index) recursion tiles
  InstDev* d_inst = nullptr;
  int2* d_cmap = nullptr;
  int4* d_tmap = nullptr;
  double* d_opart = nullptr;  // Omega partial sums [ninst][ceil(M/256)]
  int M = 0, k = 0;
  bool fp32 = false;
  int Pf = 1, Pa = 1;         // probes per wave, forward and adjoint kernels
  int Sf = -1, Sa = -1;       // block schedules (KPM_SCHED_*), -1 = the kernel's default
  bool want_tune = false;     // single lattice, automatic block, shape not tuned yet
  int4 bal = make_int4(0, 0, 0, 0);   // balanced adjoint split (blocks, probes per group,
                                      // slices per group, groups); blocks = 0: not used
  int Rmax = 0;
  long long sites = 0;
  int nrf() const { return (Rmax + kWaves * Pf - 1) / (kWaves * Pf); }
  int nra() const { return (Rmax + kWaves * Pa - 1) / (kWaves * Pa); }
  int nch() const { return (int)cmap.size(); }
  int ntl() const { return (int)tmap.size(); }
  // tiles per lattice row for a single lattice (blocks compute their tile), 0 for a batch
  int tpx() const { return inst.size() == 1 ? (inst[0].Lx + kTX - 1) / kTX : 0; }
};

void finish_ctx(Ctx& c) {
  c.cmap.clear();
  c.tmap.clear();
  c.Rmax = 0;
  c.sites = 0;
  for (size_t q = 0; q < c.inst.size(); ++q) {
    const InstDev& I = c.inst[q];
    for (int ch = 0; ch * kBlock < I.N; ++ch) c.cmap.push_back(make_int2((int)q, ch * kBlock));
    const int tx = (I.Lx + kTX - 1) / kTX, ty = (I.Ly + kTY - 1) / kTY;
    for (int t = 0; t < tx * ty; ++t) c.tmap.push_back(make_int4((int)q, (t % tx) * kTX, (t / tx) * kTY, t));
    c.Rmax = std::max(c.Rmax, I.R);
    c.sites += I.N;
  }
}

// compute units of the current device (0 if unknown)
int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cus;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cus.find(dev);
  if (it != cus.end()) return it->second;
  hipDeviceProp_t prop{};
  const int n = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 0;
  return cus[dev] = n;
}

// Work split of the balanced adjoint schedule (single lattice, see
// adj_bal_body): the grid is the number of blocks the chip holds at once
// (a multiple of 8, capped so that every share has at least 8 units); the
// probes form 2 groups when R is even (the XCDs then split the probes in
// halves, as in the ranges schedule), else 1; the slices per group are the
// most blocks that touch one (group, tile) segment.  Not used (bal.x = 0)
// when those slices would not fit the partial-sum buffer (ceil(R / 4)
// slices) or the lattice is too small to fill the grid.
void set_bal(Ctx& c) {
  c.bal = make_int4(0, 0, 0, 0);
  if (c.Sa != KPM_SCHED_BALANCED || c.inst.size() != 1) return;
  InstDev& I = c.inst[0];
  int nb = 0;
  if (adj_bal_blocks_per_cu(c.fp32, &nb) != hipSuccess || nb < 1) return;
  const long long cus = device_cus();
  const long long ntiles = c.ntl(), W = ntiles * I.R;
  if (W >= (1LL << 31)) return;                 // the kernel's unit indices are 32-bit
  long long G = std::min((long long)nb * cus, W / 8);
  G -= G % 8;
  if (G < 8) return;
  const int ng = I.R % 2 == 0 ? 2 : 1;
  const long long Lg = I.R / ng;
  long long S = 0;
  for (long long seg = 0; seg < ng * ntiles; ++seg) {
    // blocks holding the segment's first and last units: block_of(v) = ((v + 1) G - 1) / W
    const long long b0 = ((seg * Lg + 1) * G - 1) / W, b1 = ((seg + 1) * Lg * G - 1) / W;
    S = std::max(S, b1 - b0 + 1);
  }
  if (ng * S > (I.R + kWaves - 1) / kWaves) return;
  c.bal = make_int4((int)G, (int)Lg, (int)S, ng);
  I.npb = (int)(ng * S);
}

// number of probe ranges of each instance in the adjoint (partial dOmega/dH~
// buffers); the balanced schedule's slices instead when it applies
void set_npb(Ctx& c) {
  for (auto& I : c.inst) I.npb = (I.R + kWaves * c.Pa - 1) / (kWaves * c.Pa);
  set_bal(c);
}

// Host copies of the tables uploaded for single-lattice calls, kept alive per
// workspace so that an asynchronous copy never reads freed host memory.  Each
// entry records an event after its copies; the store keeps at most
// kMaxTables workspaces, and an entry is dropped (oldest use first) only
// after its event has completed.
struct HostTables {
  std::vector<InstDev> inst;
  std::vector<int2> cmap;
  std::vector<int4> tmap;
  hipEvent_t done = nullptr;
  unsigned long long last_use = 0;
};
std::map<const void*, HostTables> g_tables;
std::mutex g_tables_mu;
unsigned long long g_tables_clock = 0;
constexpr size_t kMaxTables = 16;

// Drops the least recently used entries beyond kMaxTables (never `keep`).
int prune_tables(const void* keep) {
  while (g_tables.size() > kMaxTables) {
    auto victim = g_tables.end();
    for (auto it = g_tables.begin(); it != g_tables.end(); ++it)
      if (it->first != keep && (victim == g_tables.end() || it->second.last_use < victim->second.last_use))
        victim = it;
    if (victim == g_tables.end()) break;
    if (victim->second.done) {
      KPM_HIP(hipEventSynchronize(victim->second.done));
      (void)hipEventDestroy(victim->second.done);
    }
    g_tables.erase(victim);
  }
  return KPM_OK;
}

int upload_from(const std::vector<InstDev>& inst, const std::vector<int2>& cmap,
                const std::vector<int4>& tmap, InstDev* d_inst, int2* d_cmap, int4* d_tmap,
                hipStream_t s) {
  KPM_HIP(hipMemcpyAsync(d_inst, inst.data(), sizeof(InstDev) * inst.size(),
                         hipMemcpyHostToDevice, s));
  KPM_HIP(hipMemcpyAsync(d_cmap, cmap.data(), sizeof(int2) * cmap.size(), hipMemcpyHostToDevice,
                         s));
  KPM_HIP(hipMemcpyAsync(d_tmap, tmap.data(), sizeof(int4) * tmap.size(), hipMemcpyHostToDevice,
                         s));
  return KPM_OK;
}

// Plans own their tables (Ctx lives as long as the plan).
int upload(Ctx& c, hipStream_t s) {
  return upload_from(c.inst, c.cmap, c.tmap, c.d_inst, c.d_cmap, c.d_tmap, s);
}

// Single-lattice calls: copy the tables into the per-workspace host store first.
// extra: instances uploaded after the lattice's own (the probe halves).
int upload_single(Ctx& c, const void* ws, hipStream_t s, const std::vector<InstDev>* extra = nullptr) {
  std::lock_guard<std::mutex> lk(g_tables_mu);
  HostTables& t = g_tables[ws];
  // the previous upload from this store may still be reading it
  if (t.done) KPM_HIP(hipEventSynchronize(t.done));
  else KPM_HIP(hipEventCreateWithFlags(&t.done, hipEventDisableTiming));
  t.inst = c.inst;
  if (extra) t.inst.insert(t.inst.end(), extra->begin(), extra->end());
  t.cmap = c.cmap;
  t.tmap = c.tmap;
  t.last_use = ++g_tables_clock;
  int st = upload_from(t.inst, t.cmap, t.tmap, c.d_inst, c.d_cmap, c.d_tmap, s);
  if (st != KPM_OK) return st;
  KPM_HIP(hipEventRecord(t.done, s));
  return prune_tables(ws);
}

int run_forward(const Ctx& c, bool ckpt, int nsteps, hipStream_t s) {
  const int ninst = (int)c.inst.size();
  hipLaunchKernelGGL(k_set_status, dim3((ninst + 63) / 64), dim3(64), 0, s, c.d_inst, ninst, 0);
  KPM_HIP(hipGetLastError());
  KPM_HIP(launch_rescale(c.d_inst, c.d_tmap, c.ntl(), c.fp32, s));
  KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, 0, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), 0, c.M, c.k,
                      ckpt ? 1 : 0, c.bal, s));
  for (int m = 0; m + 1 < nsteps; ++m)
    KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, 1, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), m, c.M, c.k,
                        ckpt ? 1 : 0, c.bal, s));
  return KPM_OK;
}

int run_moments(const Ctx& c, double* mu_user, hipStream_t s) {
  int maxRM = 0;
  for (auto& I : c.inst) maxRM = std::max(maxRM, I.R * c.M);
  KPM_HIP(launch_mom_reduce(c.d_inst, (int)c.inst.size(), maxRM, c.M, mu_user, s));
  return KPM_OK;
}

// gamma_{M-1}, gamma_{M-2} and cleared partial sums (every slice the
// balanced schedule uses; the other schedules' init clears its own ranges)
int adj_init(const Ctx& c, hipStream_t s) {
  if (c.bal.x > 0) {
    const InstDev& I = c.inst[0];
    KPM_HIP(launch_zero2(I.gpart, (long long)I.npb * kNent * I.N, s));
  }
  KPM_HIP(launch_cheb(c.fp32, c.Pa, c.Sa, 2, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nra(), 0, c.M, c.k, 0,
                      c.bal, s));
  return KPM_OK;
}

int run_adjoint(const Ctx& c, hipStream_t s) {
  const int M = c.M;
  int st = adj_init(c, s);
  if (st != KPM_OK) return st;
  for (int m = M - 3; m >= 0; --m)
    KPM_HIP(launch_cheb(c.fp32, c.Pa, c.Sa, 3, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nra(), m, M, c.k, 0, c.bal, s));
  KPM_HIP(launch_cheb(c.fp32, c.Pa, c.Sa, 3, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nra(), 0, M, c.k, 1, c.bal, s));
  KPM_HIP(launch_rho(c.d_inst, c.d_cmap, c.nch(), s));
  return KPM_OK;
}

// ------------------------------------------------------------ single lattice
// Workspace = [InstDev x 3][cmap][tmap][instance buffers]: the lattice's
// instance, then the instances of its two probe halves (see Halves).
struct WsLayout {
  size_t off_inst, off_cmap, off_tmap, off_buf, total;
};

WsLayout ws_layout(const Sizes& z) {
  WsLayout w{};
  size_t o = 0;
  w.off_inst = o; o = align_up(o + 3 * sizeof(InstDev));
  w.off_cmap = o; o = align_up(o + sizeof(int2) * z.nchunk);
  w.off_tmap = o; o = align_up(o + sizeof(int4) * z.ntile);
  w.off_buf = o;  o += inst_bytes(z);
  w.total = o;
  return w;
}

struct FwdSig {
  const double* h;
  const double* ab;
  const double* C;
  int M, R, prec, k;
  bool consumed;   // an adjoint has run: the alpha ping-pong holds alpha_0, alpha_1
  bool split;      // the forward ran as two probe halves (their buffer layout)
};
std::map<const void*, FwdSig> g_fwd;

// Puts alpha_{M-2} and alpha_{M-1} back into the ping-pong buffers after an
// adjoint pass has run them down to alpha_0: copy the last stored checkpoint
// pair (alpha_j0, alpha_j0+1), j0 = k floor((M-2)/k), and run the forward
// steps j0+1 .. M-2 again (fewer than k steps; their moment partials are
// rewritten with the same values and not reduced again).
int restore_alpha(const Ctx& c, hipStream_t s) {
  const InstDev& I = c.inst[0];
  const int M = c.M, k = c.k;
  const int j0 = ((M - 2) / k) * k;
  const size_t vec = (size_t)I.R * I.N * (c.fp32 ? 16 : 32);
  const char* ck = static_cast<const char*>(I.ckpt);
  const size_t slot = 2 * (size_t)(j0 / k);
  KPM_HIP(hipMemcpyAsync(I.A[j0 & 1], ck + slot * vec, vec, hipMemcpyDeviceToDevice, s));
  KPM_HIP(hipMemcpyAsync(I.A[(j0 + 1) & 1], ck + (slot + 1) * vec, vec, hipMemcpyDeviceToDevice, s));
  for (int m = j0 + 1; m + 1 < M; ++m)
    KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, 1, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), m, M, k, 0, c.bal, s));
  return KPM_OK;
}

// ---- autotuner: probe block and block schedule of each recursion kernel
struct Tune {
  int Pf, Sf, Pa, Sa;
};
std::map<std::string, Tune> g_tune_cache;   // this process's picks, by shape key
std::set<std::string> g_tune_miss;          // keys the file did not hold when last read

// Shape key: device (architecture, compute units), precision and every
// instance's N and R, in plan order.  A step's cost does not depend on M or
// on the checkpoint interval, so those are not part of it.
std::string device_tag() {
  static std::mutex mu;
  static std::map<int, std::string> tags;   // device ordinal -> "<arch>:<compute units>"
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "dev:0";
  std::lock_guard<std::mutex> lk(mu);
  auto it = tags.find(dev);
  if (it != tags.end()) return it->second;
  hipDeviceProp_t prop{};
  std::string arch = "dev";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return tags[dev] = arch + ":" + std::to_string(cus);
}

std::string shape_key(const Ctx& c) {
  std::string key = device_tag() + (c.fp32 ? ":f" : ":d");
  for (size_t q = 0; q < c.inst.size(); ++q)
    key += (q ? "," : ":") + std::to_string(c.inst[q].N) + "x" + std::to_string(c.inst[q].R);
  return key;
}

// On-disk cache: the file named by KPM_TUNE_CACHE, else
// $XDG_CACHE_HOME/kpm_tune.txt, else $HOME/.cache/kpm_tune.txt.  One line per
// shape: "<key> <Pf> <Sf> <Pa> <Sa>"; the last line of a key wins; lines that
// do not parse, or hold values the launchers do not take, are ignored.
std::string tune_path() {
  if (const char* e = std::getenv("KPM_TUNE_CACHE")) return e;
  if (const char* x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/kpm_tune.txt";
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/kpm_tune.txt";
  return "";
}

bool valid_tune(const Tune& t) {
  auto okP = [](int P) { return P == 1 || P == 2 || P == 4 || P == 8 || P == 16 || P == 32; };
  auto okS = [](int S) { return S >= KPM_SCHED_TILE_MAJOR && S <= KPM_SCHED_BALANCED; };
  return okP(t.Pf) && okP(t.Pa) && okS(t.Sf) && okS(t.Sa);
}

std::mutex g_tune_file_mu;   // one reader or writer of the cache file at a time in this process

bool disk_lookup(const std::string& key, Tune& out) {
  const std::string path = tune_path();
  std::lock_guard<std::mutex> lk(g_tune_file_mu);
  if (path.empty()) return false;
  std::ifstream f(path);
  if (!f) return false;
  bool found = false;
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string k;
    Tune t{};
    if (!(ls >> k >> t.Pf >> t.Sf >> t.Pa >> t.Sa)) continue;
    if (k == key && valid_tune(t)) {
      out = t;
      found = true;
    }
  }
  return found;
}

void disk_store(const std::string& key, const Tune& t) {
  const std::string path = tune_path();
  if (path.empty()) return;
  std::lock_guard<std::mutex> lk(g_tune_file_mu);
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
  std::ofstream f(path, std::ios::app);
  if (f) f << key << ' ' << t.Pf << ' ' << t.Sf << ' ' << t.Pa << ' ' << t.Sa << '\n';
}

// Picks for this shape from the process cache, else from the file (then
// remembered in the process); *source = 1 or 2.  A key the file did not hold
// is not looked up in the file again by this process.
bool tune_lookup(const std::string& key, Tune& t, int* source) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      t = it->second;
      *source = 1;
      return true;
    }
    if (g_tune_miss.count(key)) return false;
  }
  const bool hit = disk_lookup(key, t);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!hit) {
    g_tune_miss.insert(key);
    return false;
  }
  g_tune_cache[key] = t;
  *source = 2;
  return true;
}

void apply_tune(Ctx& c, const Tune& t) {
  c.Pf = t.Pf;
  c.Sf = t.Sf;
  c.Pa = t.Pa;
  c.Sa = t.Sa;
  set_npb(c);
}

// Times up to 16 plain forward steps and 16 adjoint steps for each candidate
// (probe block, schedule), the faster of two runs after a warm-up one, and
// keeps the fastest candidate of each kernel.  The rescaled rows, alpha_0
// and alpha_1 are set before the timed forward steps, so that a candidate's
// time holds the step kernel alone (with them inside, 8 timed steps picked a
// forward schedule 3 % slower than the best on the 100 x 100 workload).  The
// forward runs on the probes (the adjoint after it, on the alpha just
// computed, with gamma and the partial sums from k_adj_init), so no step
// reads uninitialised data.  KPM_TUNE_VERBOSE=1 prints every timing on stderr.
// single_ws: the workspace of a single-lattice call (its tables are uploaded
// through the per-workspace host store), or null for a plan.
int tune_ctx(Ctx& c, const void* single_ws, hipStream_t s, int* source) {
  const std::string key = shape_key(c);
  Tune t{};
  auto put = [&](Ctx& cc) { return single_ws ? upload_single(cc, single_ws, s) : upload(cc, s); };
  if (tune_lookup(key, t, source)) {
    apply_tune(c, t);
    return put(c);
  }
  const bool verbose = std::getenv("KPM_TUNE_VERBOSE") != nullptr;
  // timing events, destroyed on every return path
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  KPM_HIP(hipEventCreate(&ev.a));
  KPM_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  // adjoint: `steps` launches at m = M-3; forward: the plain steps m = fm0 .. fm1
  // (alpha_0, alpha_1 and the rescaled rows are set first, untimed)
  const int steps = std::min(c.M, 16);
  const int fm0 = c.M >= 3 ? 1 : 0, fm1 = std::min(c.M - 2, fm0 + 15);
  float best_f = 1e30f, best_a = 1e30f;
  Tune best{1, -1, 1, -1};
  int st = KPM_OK;
  for (int P : {1, 2, 4, 8, 16, 32}) {
    for (int S : {KPM_SCHED_TILE_MAJOR, KPM_SCHED_RANGES, KPM_SCHED_STRIPS, KPM_SCHED_STRIP_TILES,
                  KPM_SCHED_BALANCED}) {
      // the balanced adjoint does not depend on the probe block (the forward
      // then runs its default schedule): one candidate is enough
      if (S == KPM_SCHED_BALANCED && P != 32) continue;
      c.Pf = c.Pa = P;
      c.Sf = c.Sa = S;
      set_npb(c);
      if ((st = put(c)) != KPM_OK) break;
      // forward: warm once, then the faster of two timed runs
      if ((st = run_forward(c, true, fm0 + 1, s)) != KPM_OK) break;
      float tf = 1e30f;
      for (int rep = 0; rep < 3 && st == KPM_OK; ++rep) {
        KPM_HIP(hipEventRecord(e0, s));
        for (int m = fm0; m <= fm1; ++m)
          KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, 1, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), m, c.M,
                              c.k, 1, c.bal, s));
        KPM_HIP(hipEventRecord(e1, s));
        KPM_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        KPM_HIP(hipEventElapsedTime(&t, e0, e1));
        if (rep > 0) tf = std::min(tf, t);
      }
      if (st != KPM_OK) break;
      if (tf < best_f && S != KPM_SCHED_BALANCED) {
        best_f = tf;
        best.Pf = P;
        best.Sf = S;
      }
      float ta = 1e30f;
      if (c.M >= 3) {
        // adjoint steps at m = M-3 (timing only) on initialised data: alpha from the
        // forward steps just timed (with checkpoint stores, so an anchored step at
        // small M reads written slots), gamma and the partial sums from k_adj_init;
        // warm once, then the faster of two timed runs
        if ((st = adj_init(c, s)) != KPM_OK) break;
        for (int rep = 0; rep < 3; ++rep) {
          KPM_HIP(hipEventRecord(e0, s));
          for (int q = 0; q < steps; ++q)
            KPM_HIP(launch_cheb(c.fp32, c.Pa, c.Sa, 3, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nra(),
                                c.M - 3, c.M, c.M + 1, 0, c.bal, s));
          KPM_HIP(hipEventRecord(e1, s));
          KPM_HIP(hipEventSynchronize(e1));
          float t = 0.f;
          KPM_HIP(hipEventElapsedTime(&t, e0, e1));
          if (rep > 0) ta = std::min(ta, t);
        }
        if (ta < best_a) {
          best_a = ta;
          best.Pa = P;
          best.Sa = S;
        }
      }
      if (verbose)
        std::fprintf(stderr, "[kpm tune] %s P=%d sched=%d forward %.1f us/step adjoint %.1f us/step\n",
                     key.c_str(), P, S, 1e3f * tf / (fm1 - fm0 + 1), 1e3f * ta / steps);
    }
    if (st != KPM_OK) break;
  }
  if (st != KPM_OK) return st;
  *source = 0;
  if (c.M < 3) {
    // no adjoint step to time: use the forward's pick, and remember nothing
    best.Pa = best.Pf;
    best.Sa = best.Sf;
    apply_tune(c, best);
    return put(c);
  }
  apply_tune(c, best);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune_cache[key] = best;
  }
  disk_store(key, best);
  return put(c);
}


int prepare_single(Ctx& c, const kpm_lattice* L, const double* h, const double* ab,
                   const kpm_probes* pr, int M, const double* C, int prec, int k, void* ws,
                   size_t ws_bytes, bool fwd_only = false) {
  if (!valid_lattice(L) || !h || !ab || !ws) return KPM_EINVAL;
  if (M < 2 || k < 2) return KPM_EINVAL;
  if (prec != KPM_FP64 && prec != KPM_FP32) return KPM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return KPM_EINVAL;
  InstDev I;
  std::memset(&I, 0, sizeof(I));
  int ng = 0;
  const int R = build_groups(L, pr, I.g, &ng);
  if (R < 1 || !records_fit(L, R)) return KPM_EINVAL;
  c.fp32 = prec == KPM_FP32;
  const Sizes z = sizes(L, R, M, k, c.fp32, fwd_only);
  const WsLayout w = ws_layout(z);
  if (ws_bytes < w.total) return KPM_EWORKSPACE;
  char* base = static_cast<char*>(ws);
  I.Lx = L->Lx;
  I.Ly = L->Ly;
  I.N = z.N;
  I.R = R;
  I.nchunk = z.ntile;
  I.ngroups = ng;
  I.h = reinterpret_cast<const double2*>(h);
  I.ab = ab;
  I.C = C;
  carve(I, z, base + w.off_buf);
  c.inst.assign(1, I);
  c.d_inst = reinterpret_cast<InstDev*>(base + w.off_inst);
  c.d_cmap = reinterpret_cast<int2*>(base + w.off_cmap);
  c.d_tmap = reinterpret_cast<int4*>(base + w.off_tmap);
  c.M = M;
  c.k = k;
  finish_ctx(c);
  int P;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    P = g_probe_block;
    c.Sf = g_sched_f;
    c.Sa = g_sched_a;
  }
  c.Pf = P ? P : auto_probe_fwd(c.ntl(), c.Rmax);
  c.Pa = P ? P : auto_probe_adj(c.ntl(), c.Rmax);
  set_npb(c);
  // the forward-only layout (the entry point without allocation) keeps the
  // size heuristic: no cache lookup, no file access
  if (P == 0 && !fwd_only) {
    Tune t{};
    int src = 0;
    if (tune_lookup(shape_key(c), t, &src)) apply_tune(c, t);
    else c.want_tune = true;
  }
  return KPM_OK;
}

// First forward of a shape with the automatic probe block: time the
// candidates on this call's workspace (whose state the forward then rebuilds;
// a forward kept for a later gradient is forgotten first).  Not while the
// stream is being captured: the timing synchronises.
int tune_single(Ctx& c, const void* ws, hipStream_t s) {
  if (!c.want_tune) return KPM_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  KPM_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return KPM_OK;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_fwd.erase(ws);
  }
  int src = 0;
  int st = tune_ctx(c, ws, s, &src);
  c.want_tune = false;
  return st;
}

// ------------------------------------------------------------ probe halves
// The probes of a single lattice can run as two halves on two streams, the
// caller's and a second one per device, with their step launches
// interleaved.  A launch of one half leaves block slots idle while its last
// blocks finish, and the other half's blocks take them; each half keeps the
// probe lockstep of its own blocks.  Measured on the 100 x 100 workload
// (M = 4096, 256 probes, FP32): 281 ms per energy + gradient for two
// 128-probe halves side by side, 308 ms for the 256 probes on one stream.
//
// A half is an instance over its contiguous share of the probe-indexed
// buffers: probes [poff, poff + R_h) of the vectors, code table, weights and
// reduced moments; its own [S][R_h][N] share of the checkpoints and
// [M][ntile][R_h] share of the moment partials; its own partial-sum slices
// (half 1's after half 0's).  The lattice's instance then reduces over both:
// Omega over all moments, rho over all slices.
int g_streams = 0;                  // 0 automatic, 1 one stream, 2 probe halves

struct Halves {
  bool on = false;
  Ctx h[2];
  std::vector<InstDev> inst() const { return {h[0].inst[0], h[1].inst[0]}; }
};

// The second stream of the current device (created once, default priority).
int secondary_stream(hipStream_t* out) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  KPM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it == streams.end()) {
    hipStream_t st = nullptr;
    KPM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    it = streams.emplace(dev, st).first;
  }
  *out = it->second;
  return KPM_OK;
}

// Whether a call runs as probe halves: requested (kpm_set_streams(2)), or
// automatically when each half still keeps the chip busy: R >= 128 and
// R N >= 2^19 site-probes.  Measured (ms per energy + gradient, one stream
// against halves): 100 x 100, R = 256, 75.8 / 69.3 (FP32) and 177.7 / 170.5
// (FP64) at M = 1024; 48 x 96, R = 128, 26.0 / 24.1 (and 26.0 / 24.6 per
// evaluation inside the self-consistent loop); 64 x 64, R = 192,
// 60.7 / 59.1; 32 x 32, R = 2048, 16.8 / 16.8; but 64 x 64, R = 64,
// 15.3 / 17.0.  Never while the stream is being captured.
bool split_wanted(const Ctx& c, hipStream_t s) {
  int mode;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    mode = g_streams;
  }
  const InstDev& F = c.inst[0];
  if (mode == 1 || F.R < 2) return false;
  if (mode == 0 && (F.R < 128 || (long long)F.R * F.N < (1LL << 19))) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
}

// The two half contexts of c (ceil(R/2) and floor(R/2) probes) with c's probe
// blocks and schedules; false (hv.on stays false) when their partial-sum
// slices do not fit the lattice's buffer (gpart_slices).
bool build_halves(Ctx& c, Halves& hv) {
  hv.on = false;
  const InstDev& F = c.inst[0];
  const int R0 = (F.R + 1) / 2;
  const size_t rec = c.fp32 ? 16 : 32;
  const size_t nslots = 2 * (size_t)((c.M - 1) / c.k + 1);
  for (int q = 0; q < 2; ++q) {
    Ctx& h = hv.h[q];
    h = c;
    h.want_tune = false;
    InstDev& I = h.inst[0];
    const size_t off = q ? R0 : 0;
    I.R = q ? F.R - R0 : R0;
    I.poff = (int)off;
    for (int j = 0; j < 2; ++j) {
      I.A[j] = static_cast<char*>(F.A[j]) + off * F.N * rec;
      I.G[j] = static_cast<char*>(F.G[j]) + off * F.N * rec;
    }
    I.ckpt = static_cast<char*>(F.ckpt) + nslots * off * F.N * rec;
    I.mom = F.mom + (size_t)c.M * F.nchunk * off;
    I.musum = F.musum + off * c.M;
    I.pcode = F.pcode + off * F.N;
    I.pw = F.pw + off;
    h.Rmax = I.R;
    h.d_inst = c.d_inst + 1 + q;
    set_npb(h);
  }
  const int npb0 = hv.h[0].inst[0].npb, npb1 = hv.h[1].inst[0].npb;
  if (npb0 + npb1 > gpart_slices(F.R)) return false;
  hv.h[1].inst[0].gpart = F.gpart + (size_t)npb0 * kNent * F.N;
  c.inst[0].npb = npb0 + npb1;
  hv.on = true;
  return true;
}

// Fork/join between the caller's stream and the second stream; while forked,
// the second stream's launches are not timed by the profiler.
struct Fork {
  hipStream_t s2 = nullptr;
  hipEvent_t e = nullptr;
  ~Fork() {
    profile_secondary(nullptr);
    if (e) (void)hipEventDestroy(e);
  }
};

int fork_from(Fork& f, hipStream_t s) {
  const int st = secondary_stream(&f.s2);
  if (st != KPM_OK) return st;
  KPM_HIP(hipEventCreateWithFlags(&f.e, hipEventDisableTiming));
  KPM_HIP(hipEventRecord(f.e, s));
  KPM_HIP(hipStreamWaitEvent(f.s2, f.e, 0));
  profile_secondary(f.s2);
  return KPM_OK;
}

int join_to(Fork& f, hipStream_t s) {
  profile_secondary(nullptr);
  KPM_HIP(hipEventRecord(f.e, f.s2));
  KPM_HIP(hipStreamWaitEvent(s, f.e, 0));
  return KPM_OK;
}

// Forward recursion of both halves (alpha_0 ... alpha_{M-1}), then their
// moment reductions (mu_user: the caller's [R][M] copy, or null; probe
// halves of a single lattice only).  c: the whole call (one lattice, or all
// instances of a batch), whose status words and rescaled rows are set here.
int run_forward_split(const Ctx& c, const Halves& hv, bool ckpt, double* mu_user, hipStream_t s,
                      int nsteps = -1, bool moments = true) {
  if (nsteps < 0) nsteps = c.M;
  const int ninst = (int)c.inst.size();
  hipLaunchKernelGGL(k_set_status, dim3((ninst + 63) / 64), dim3(64), 0, s, c.d_inst, ninst, 0);
  KPM_HIP(hipGetLastError());
  KPM_HIP(launch_rescale(c.d_inst, c.d_tmap, c.ntl(), c.fp32, s));
  Fork f;
  int st = fork_from(f, s);
  if (st != KPM_OK) return st;
  const hipStream_t ss[2] = {s, f.s2};
  for (int q = 0; q < 2; ++q) {
    const Ctx& h = hv.h[q];
    KPM_HIP(launch_cheb(h.fp32, h.Pf, h.Sf, 0, h.d_inst, h.d_tmap, h.ntl(), h.tpx(), h.nrf(), 0, h.M, h.k,
                        ckpt ? 1 : 0, h.bal, ss[q]));
  }
  for (int m = 0; m + 1 < nsteps; ++m)
    for (int q = 0; q < 2; ++q) {
      const Ctx& h = hv.h[q];
      KPM_HIP(launch_cheb(h.fp32, h.Pf, h.Sf, 1, h.d_inst, h.d_tmap, h.ntl(), h.tpx(), h.nrf(), m, h.M,
                          h.k, ckpt ? 1 : 0, h.bal, ss[q]));
    }
  if ((st = join_to(f, s)) != KPM_OK) return st;
  for (int q = 0; q < 2 && moments; ++q) {
    const Ctx& h = hv.h[q];
    double* mu = mu_user ? mu_user + (size_t)h.inst[0].poff * c.M : nullptr;
    if ((st = run_moments(h, mu, s)) != KPM_OK) return st;
  }
  return KPM_OK;
}

// Adjoint of both halves into their partial-sum slices, then rho from all slices.
int run_adjoint_split(const Ctx& c, const Halves& hv, hipStream_t s) {
  Fork f;
  int st = fork_from(f, s);
  if (st != KPM_OK) return st;
  const hipStream_t ss[2] = {s, f.s2};
  for (int q = 0; q < 2; ++q)
    if ((st = adj_init(hv.h[q], ss[q])) != KPM_OK) return st;
  for (int m = c.M - 3; m >= 0; --m)
    for (int q = 0; q < 2; ++q) {
      const Ctx& h = hv.h[q];
      KPM_HIP(launch_cheb(h.fp32, h.Pa, h.Sa, 3, h.d_inst, h.d_tmap, h.ntl(), h.tpx(), h.nra(), m, h.M, h.k,
                          0, h.bal, ss[q]));
    }
  for (int q = 0; q < 2; ++q) {
    const Ctx& h = hv.h[q];
    KPM_HIP(launch_cheb(h.fp32, h.Pa, h.Sa, 3, h.d_inst, h.d_tmap, h.ntl(), h.tpx(), h.nra(), 0, h.M, h.k, 1,
                        h.bal, ss[q]));
  }
  if ((st = join_to(f, s)) != KPM_OK) return st;
  KPM_HIP(launch_rho(c.d_inst, c.d_cmap, c.nch(), s));
  return KPM_OK;
}

constexpr int kNoFit = 1;   // a candidate whose halves do not fit (tune_pair)

// Tuning of two halves that run side by side (the probe halves of a single
// lattice, the instance halves of a batch plan).  Each candidate is timed on
// both halves at once, the same candidate for both, with their step launches
// interleaved on the caller's stream and the second stream as the calls run
// them; a half timed alone can favour a block that the pair runs slower
// (forward probe block 8 against 16 on the 48-lattice batch: 264.5 against
// 259.4 ms per energy + gradient).  Candidates, timing and the kept picks as
// in tune_ctx; the picks are remembered under `key`.  c: the whole call,
// whose status words and rescaled rows the timed forward sets.  prep(t) sets
// candidate t on both halves and uploads the tables: KPM_OK, kNoFit (the
// candidate is skipped) or an error.  With a remembered pick, or after the
// timing, the pick is left set; with neither (allow_timing false), nothing
// changes.
template <typename Prep>
int tune_pair(Ctx& c, Halves& hv, const std::string& key, Prep prep, hipStream_t s, bool allow_timing,
              int* source) {
  Tune t{};
  if (tune_lookup(key, t, source)) {
    const int r = prep(t);
    return r == kNoFit ? KPM_OK : r;
  }
  if (!allow_timing) return KPM_OK;
  const bool verbose = std::getenv("KPM_TUNE_VERBOSE") != nullptr;
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  KPM_HIP(hipEventCreate(&ev.a));
  KPM_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  auto elapsed = [&](float* ms) -> int {
    KPM_HIP(hipEventSynchronize(e1));
    KPM_HIP(hipEventElapsedTime(ms, e0, e1));
    return KPM_OK;
  };
  const int steps = std::min(c.M, 16);
  const int fm0 = c.M >= 3 ? 1 : 0, fm1 = std::min(c.M - 2, fm0 + 15);
  float best_f = 1e30f, best_a = 1e30f;
  Tune best{1, -1, 1, -1};
  bool any = false;
  int st = KPM_OK;
  for (int P : {1, 2, 4, 8, 16, 32}) {
    for (int S : {KPM_SCHED_TILE_MAJOR, KPM_SCHED_RANGES, KPM_SCHED_STRIPS, KPM_SCHED_STRIP_TILES,
                  KPM_SCHED_BALANCED}) {
      if (S == KPM_SCHED_BALANCED && P != 32) continue;
      const int r = prep(Tune{P, S, P, S});
      if (r == kNoFit) continue;
      if ((st = r) != KPM_OK) break;
      any = true;
      // forward steps of both halves (alpha_0, alpha_1 and the rescaled rows
      // set first, untimed): warm once, then the faster of two timed runs
      if ((st = run_forward_split(c, hv, true, nullptr, s, fm0 + 1, false)) != KPM_OK) break;
      float tf = 1e30f;
      for (int rep = 0; rep < 3 && st == KPM_OK; ++rep) {
        KPM_HIP(hipEventRecord(e0, s));
        {
          Fork f;
          if ((st = fork_from(f, s)) != KPM_OK) break;
          const hipStream_t ss[2] = {s, f.s2};
          for (int mm = fm0; mm <= fm1; ++mm)
            for (int q = 0; q < 2; ++q) {
              const Ctx& h = hv.h[q];
              KPM_HIP(launch_cheb(h.fp32, h.Pf, h.Sf, 1, h.d_inst, h.d_tmap, h.ntl(), h.tpx(), h.nrf(), mm,
                                  h.M, h.k, 1, h.bal, ss[q]));
            }
          if ((st = join_to(f, s)) != KPM_OK) break;
        }
        KPM_HIP(hipEventRecord(e1, s));
        float ms = 0.f;
        if ((st = elapsed(&ms)) != KPM_OK) break;
        if (rep > 0) tf = std::min(tf, ms);
      }
      if (st != KPM_OK) break;
      if (tf < best_f && S != KPM_SCHED_BALANCED) {
        best_f = tf;
        best.Pf = P;
        best.Sf = S;
      }
      float ta = 1e30f;
      if (c.M >= 3) {
        // adjoint steps of both halves at m = M-3 (timing only) on the alpha
        // just computed, gamma and the partial sums from k_adj_init
        for (int q = 0; q < 2 && st == KPM_OK; ++q) st = adj_init(hv.h[q], s);
        for (int rep = 0; rep < 3 && st == KPM_OK; ++rep) {
          KPM_HIP(hipEventRecord(e0, s));
          {
            Fork f;
            if ((st = fork_from(f, s)) != KPM_OK) break;
            const hipStream_t ss[2] = {s, f.s2};
            for (int i = 0; i < steps; ++i)
              for (int q = 0; q < 2; ++q) {
                const Ctx& h = hv.h[q];
                KPM_HIP(launch_cheb(h.fp32, h.Pa, h.Sa, 3, h.d_inst, h.d_tmap, h.ntl(), h.tpx(), h.nra(),
                                    h.M - 3, h.M, h.M + 1, 0, h.bal, ss[q]));
              }
            if ((st = join_to(f, s)) != KPM_OK) break;
          }
          KPM_HIP(hipEventRecord(e1, s));
          float ms = 0.f;
          if ((st = elapsed(&ms)) != KPM_OK) break;
          if (rep > 0) ta = std::min(ta, ms);
        }
        if (st != KPM_OK) break;
        if (ta < best_a) {
          best_a = ta;
          best.Pa = P;
          best.Sa = S;
        }
      }
      if (verbose)
        std::fprintf(stderr, "[kpm tune] %s P=%d sched=%d forward %.1f us/step adjoint %.1f us/step (both halves)\n",
                     key.c_str(), P, S, 1e3f * tf / (fm1 - fm0 + 1), 1e3f * ta / steps);
    }
    if (st != KPM_OK) break;
  }
  if (st != KPM_OK) return st;
  if (!any) return KPM_OK;
  *source = 0;
  if (c.M < 3) {
    best.Pa = best.Pf;
    best.Sa = best.Sf;
  } else {
    {
      std::lock_guard<std::mutex> lk(g_mu);
      g_tune_cache[key] = best;
    }
    disk_store(key, best);
  }
  const int r = prep(best);
  return r == kNoFit ? KPM_OK : r;
}

// Configures the probe halves of a single lattice: with the automatic probe
// block, the picks remembered for the lattice's shape as halves, else
// (allow_timing: the first energy evaluation of the shape) tune_pair's
// timing on this call's workspace; the halves are built with those picks.
// The call runs on one stream if they no longer fit.
int setup_halves(Ctx& c, Halves& hv, const void* ws, hipStream_t s, bool allow_timing) {
  if (!build_halves(c, hv)) return KPM_OK;
  int P;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    P = g_probe_block;
  }
  if (P != 0) return KPM_OK;
  const Tune orig{c.Pf, c.Sf, c.Pa, c.Sa};
  const std::string key = shape_key(c) + "/2";
  Tune t{};
  int src = 0;
  if (!tune_lookup(key, t, &src)) {
    if (!allow_timing) return KPM_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    g_fwd.erase(ws);
  }
  auto prep = [&](const Tune& cand) -> int {
    apply_tune(c, cand);
    if (!build_halves(c, hv)) return kNoFit;
    const std::vector<InstDev> ex = hv.inst();
    return upload_single(c, ws, s, &ex);
  };
  const int st = tune_pair(c, hv, key, prep, s, allow_timing, &src);
  if (st != KPM_OK) return st;
  if (!hv.on) {
    // no pick fits as halves: the size heuristic's picks, on one stream
    apply_tune(c, orig);
    build_halves(c, hv);
  }
  c.want_tune = false;
  return KPM_OK;
}

// restore_alpha for both halves (a second adjoint after one forward).
int restore_alpha_split(const Halves& hv, hipStream_t s) {
  Fork f;
  int st = fork_from(f, s);
  if (st != KPM_OK) return st;
  if ((st = restore_alpha(hv.h[0], s)) != KPM_OK) return st;
  if ((st = restore_alpha(hv.h[1], f.s2)) != KPM_OK) return st;
  return join_to(f, s);
}

}  // namespace

// ------------------------------------------------------------ batch plans
// A plan's instances can run as two instance halves (hv.on): two contexts
// over disjoint subsets of the instances (idx[q]: positions in the plan's
// instance list, ascending), each with its own instance, chunk and tile
// tables and its own tuning, whose recursions run side by side on the
// caller's stream and on the device's second stream.  The instance buffers
// belong to the whole plan (c); a half's table holds copies of its
// instances' entries.
struct KpmBatchPlan {
  Ctx c;
  void* mem = nullptr;
  hipStream_t capture_stream = nullptr;   // graphs are captured here, launched on the caller's
  bool tuned = false;
  int tune_source = -1;                 // 0 timed, 1 process cache, 2 disk cache, -1 fixed
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<const void*> graph_ptrs;   // pointers the captured graph was built with
  Halves hv;
  std::vector<int> idx[2];
  hipStream_t capture2 = nullptr;        // capture stream of the second half's graph
  hipGraphExec_t exec2 = nullptr;
  hipGraph_t graph2 = nullptr;
  // A plan of instance groups (batch_group_count) holds one plan per group,
  // run one after another, and no instances of its own; gidx[g]: the
  // group's instances, as positions in the caller's arrays, ascending.
  std::vector<KpmBatchPlan*> groups;
  std::vector<std::vector<int>> gidx;
};

namespace {

int batch_sequence_ctx(Ctx& c, hipStream_t s) {
  int st = run_forward(c, true, c.M, s);
  if (st != KPM_OK) return st;
  if ((st = run_moments(c, nullptr, s)) != KPM_OK) return st;
  KPM_HIP(launch_omega(c.d_inst, (int)c.inst.size(), c.M, s));
  return run_adjoint(c, s);
}

int batch_sequence(KpmBatchPlan* pl, hipStream_t s) {
  if (!pl->hv.on) return batch_sequence_ctx(pl->c, s);
  // instance halves, step launches interleaved on two streams
  Ctx& c = pl->c;
  int st = run_forward_split(c, pl->hv, true, nullptr, s);
  if (st != KPM_OK) return st;
  KPM_HIP(launch_omega(c.d_inst, (int)c.inst.size(), c.M, s));
  return run_adjoint_split(c, pl->hv, s);
}

// Copies the plan's instance entries (the call's pointers, the probe range
// counts) into the halves' tables.
void sync_halves(KpmBatchPlan* pl) {
  for (int q = 0; q < 2; ++q)
    for (size_t j = 0; j < pl->idx[q].size(); ++j) pl->hv.h[q].inst[j] = pl->c.inst[pl->idx[q][j]];
}

// After a half's probe blocks changed: its instances' probe range counts
// (the partial-sum slices that k_rho adds) into the plan's entries.
void npb_from_halves(KpmBatchPlan* pl) {
  for (int q = 0; q < 2; ++q)
    for (size_t j = 0; j < pl->idx[q].size(); ++j) pl->c.inst[pl->idx[q][j]].npb = pl->hv.h[q].inst[j].npb;
}

int upload_plan(KpmBatchPlan* pl, hipStream_t s) {
  int st = upload(pl->c, s);
  if (st != KPM_OK || !pl->hv.on) return st;
  sync_halves(pl);
  for (int q = 0; q < 2 && st == KPM_OK; ++q) st = upload(pl->hv.h[q], s);
  return st;
}

// Whether a batch plan runs as instance halves: requested
// (kpm_set_streams(2)), or automatically when the instances hold
// sum R N >= 2^19 site-probes.  Measured (ms per energy + gradient, FP32,
// M = 1024, the first n of 48 lattices of 24 ... 64 sites a side with 64
// probes each, graph replays, one stream against halves): n = 2 (3.6e5
// site-probes) 19.2 / 19.3; n = 3 (5.1e5) 23.6 / 22.9; n = 4 (7.1e5)
// 28.8 / 28.5; n = 6 (9.8e5) 36.1 / 33.3; n = 12 (1.7e6) 61.2 / 50.0;
// n = 24 (3.6e6) 137.4 / 131.4; n = 48 (7.2e6) 279.7 / 264.9.
bool batch_split_wanted(const std::vector<InstDev>& inst) {
  int mode;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    mode = g_streams;
  }
  if (inst.size() < 2 || mode == 1) return false;
  long long rn = 0;
  for (const auto& I : inst) rn += (long long)I.R * I.N;
  return mode == 2 || rn >= (1LL << 19);
}

// Splits the plan's instances into two halves of nearly equal R N (largest
// first, each to the lighter half), each half in the plan's order.
void split_instances(const std::vector<InstDev>& inst, std::vector<int> idx[2]) {
  std::vector<int> order(inst.size());
  for (size_t q = 0; q < inst.size(); ++q) order[q] = (int)q;
  auto w = [&](int q) { return (long long)inst[q].R * inst[q].N; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w(a) > w(b); });
  long long load[2] = {0, 0};
  idx[0].clear();
  idx[1].clear();
  for (int q : order) {
    const int j = load[0] <= load[1] ? 0 : 1;
    idx[j].push_back(q);
    load[j] += w(q);
  }
  std::sort(idx[0].begin(), idx[0].end());
  std::sort(idx[1].begin(), idx[1].end());
}

// Instance groups of a batch plan, run one after another: kpm_set_batch_groups
// when set, else as many as keep each group's adjoint step traffic (6 passes
// of its sum R N records: alpha and gamma at m+1 and m+2 read, alpha_m and
// gamma_m written over the m+2 sets) within kGroupBytes, i.e. its 4 distinct
// vector sets within 160 MB, so that they stay in the 256 MB Infinity Cache
// from one step to the next (with the coefficients and partial sums) rather
// than streaming from HBM.  Measured (the 48 uneven lattices, FP32, M = 1024,
// 7.2e6 site-probes, 693 MB of adjoint traffic and 462 MB of distinct vectors
// per step; groups balanced by R N, each as two instance halves; ms per
// energy + gradient): 1 group 258.9, 2: 230.9 (231 MB distinct per group),
// 3: 190.9 (154 MB), 4: 201.2, 5: 212.2, 6: 225.7, 8: 241.4; in FP64 (twice
// the bytes): 1 group 527.1, 2: 516.1, 3: 472.1, 4: 464.0, 6: 450.7 (154 MB),
// 8: 464.7.
constexpr double kGroupBytes = 240e6;
int32_t g_batch_groups = 0;   // 0 automatic, else the group count (at most one per instance)

int batch_group_count(const std::vector<long long>& rn, bool fp32) {
  int fixed;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    fixed = g_batch_groups;
  }
  const int n = (int)rn.size();
  if (fixed > 0) return std::min(fixed, n);
  double total = 0.0;
  for (long long v : rn) total += (double)v;
  const double bytes = 6.0 * (fp32 ? 16.0 : 32.0) * total;
  const int G = (int)std::ceil(bytes / kGroupBytes);
  return std::max(1, std::min(G, n));
}

// Splits instances into G groups of nearly equal R N (largest first, each to
// the lightest group), each group in the plan's order.
std::vector<std::vector<int>> group_instances(const std::vector<long long>& rn, int G) {
  std::vector<int> order(rn.size());
  for (size_t q = 0; q < rn.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rn[a] > rn[b]; });
  std::vector<std::vector<int>> out(G);
  std::vector<long long> load(G, 0);
  for (int q : order) {
    const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    out[j].push_back(q);
    load[j] += rn[q];
  }
  for (auto& g : out) std::sort(g.begin(), g.end());
  return out;
}

}  // namespace

// ------------------------------------------------------------ static scratch
// Workspace of kpm_moments_noalloc: one array per GPU, held for the life of
// the process.  In host code the name is only a stand-in for the symbol; the
// device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[KPM_NOALLOC_SCRATCH_BYTES];

namespace kpm {
// Writes the instance table and the site-chunk and tile maps of a single
// lattice (as finish_ctx lays them out) into the scratch; the table travels
// as a kernel argument, so no host buffer has to outlive the call.
__global__ void k_fill_tables(InstDev I, InstDev* d_inst, int2* d_cmap, int4* d_tmap, int nchunk,
                              int ntile, int tiles_x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *d_inst = I;
  if (t < nchunk) d_cmap[t] = make_int2(0, t * kBlock);
  if (t < ntile) d_tmap[t] = make_int4(0, (t % tiles_x) * 8, (t / tiles_x) * 4, t);
}
}  // namespace kpm

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device ordinal -> address of `scratch` there

// Address of the current device's scratch, looked up once per device with
// that device current.
int scratch_address(void** out) {
  int dev = 0;
  KPM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    KPM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return KPM_EDEVICE;
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return KPM_OK;
}
}  // namespace

extern "C" {

int32_t kpm_probe_count(const kpm_lattice* lat, const kpm_probes* probes) {
  if (!valid_lattice(lat)) return KPM_EINVAL;
  int R = build_groups(lat, probes, nullptr, nullptr);
  return R < 1 ? KPM_EINVAL : R;
}

int kpm_build_H(const kpm_lattice* lat, const kpm_model* model, const double* n, const double* chi,
                const double* delta, double* h, void* stream) {
  if (!valid_lattice(lat) || !model || !n || !chi || !delta || !h) return KPM_EINVAL;
  ModelDev md{lat->Lx, lat->Ly, lat->n_vortex, lat->Lx * lat->Ly, model->t, model->tp, model->J,
              model->mu};
  KPM_HIP(launch_build_h(md, n, chi, delta, h, static_cast<hipStream_t>(stream)));
  return KPM_OK;
}

int kpm_build_H_sdw(const kpm_lattice* lat, const kpm_model* model, const double* n_up,
                    const double* n_dn, const double* chi_up, const double* chi_dn,
                    const double* delta_up, const double* delta_dn, double* h, void* stream) {
  if (!valid_lattice(lat) || !model || !n_up || !n_dn || !chi_up || !chi_dn || !delta_up ||
      !delta_dn || !h)
    return KPM_EINVAL;
  ModelDev md{lat->Lx, lat->Ly, lat->n_vortex, lat->Lx * lat->Ly, model->t, model->tp, model->J,
              model->mu};
  KPM_HIP(launch_build_sdw(md, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, h,
                           static_cast<hipStream_t>(stream)));
  return KPM_OK;
}

int kpm_build_H_sdw_vjp(const kpm_lattice* lat, const kpm_model* model, const double* n_up,
                        const double* n_dn, const double* chi_up, const double* chi_dn,
                        const double* delta_up, const double* delta_dn, const double* rho,
                        double* dn_up, double* dn_dn, double* dchi_up, double* dchi_dn,
                        double* ddelta_up, double* ddelta_dn, void* stream) {
  if (!valid_lattice(lat) || !model || !n_up || !n_dn || !chi_up || !chi_dn || !delta_up ||
      !delta_dn || !rho || !dn_up || !dn_dn || !dchi_up || !dchi_dn || !ddelta_up || !ddelta_dn)
    return KPM_EINVAL;
  ModelDev md{lat->Lx, lat->Ly, lat->n_vortex, lat->Lx * lat->Ly, model->t, model->tp, model->J,
              model->mu};
  KPM_HIP(launch_build_sdw_vjp(md, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, rho, dn_up, dn_dn,
                               dchi_up, dchi_dn, ddelta_up, ddelta_dn, static_cast<hipStream_t>(stream)));
  return KPM_OK;
}

int kpm_build_H_vjp(const kpm_lattice* lat, const kpm_model* model, const double* n,
                    const double* chi, const double* delta, const double* rho, double* dn,
                    double* dchi, double* ddelta, void* stream) {
  if (!valid_lattice(lat) || !model || !n || !chi || !delta || !rho || !dn || !dchi || !ddelta)
    return KPM_EINVAL;
  ModelDev md{lat->Lx, lat->Ly, lat->n_vortex, lat->Lx * lat->Ly, model->t, model->tp, model->J,
              model->mu};
  KPM_HIP(launch_build_vjp(md, n, chi, delta, rho, dn, dchi, ddelta,
                           static_cast<hipStream_t>(stream)));
  return KPM_OK;
}

int kpm_bounds(const kpm_lattice* lat, const double* h, double* ab, void* stream) {
  if (!valid_lattice(lat) || !h || !ab) return KPM_EINVAL;
  KPM_HIP(launch_bounds(lat->Lx, lat->Ly, h, ab, static_cast<hipStream_t>(stream)));
  return KPM_OK;
}

int kpm_coefficients(int32_t M, double T, const double* ab, int32_t K, double* C, void* stream) {
  if (M < 2 || !(T > 0.0) || !std::isfinite(T) || !ab || !C || K < 0) return KPM_EINVAL;
  if (K == 0) K = std::max(4 * M, 16384);
  if (K < M || K > (1 << 28)) return KPM_EINVAL;
  KPM_HIP(launch_coeffs(M, K, T, ab, C, static_cast<hipStream_t>(stream)));
  return KPM_OK;
}

size_t kpm_workspace_size(const kpm_lattice* lat, int32_t R, int32_t M, int32_t ckpt_k,
                          int32_t precision) {
  if (!valid_lattice(lat) || R < 1 || R > kMaxR || M < 2 || ckpt_k < 2) return 0;
  if (precision != KPM_FP64 && precision != KPM_FP32) return 0;
  return ws_layout(sizes(lat, R, M, ckpt_k, precision == KPM_FP32)).total;
}

int kpm_moments(const kpm_lattice* lat, const double* h, const double* ab, const kpm_probes* probes,
                int32_t M, int32_t precision, int32_t ckpt_k, double* mu, void* ws,
                size_t ws_bytes, void* stream) {
  if (!mu) return KPM_EINVAL;
  Ctx c;
  int st = prepare_single(c, lat, h, ab, probes, M, nullptr, precision, ckpt_k, ws, ws_bytes);
  if (st != KPM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Halves hv;
  if (split_wanted(c, s) && (st = setup_halves(c, hv, ws, s, false)) != KPM_OK) return st;
  const std::vector<InstDev> ex = hv.on ? hv.inst() : std::vector<InstDev>();
  if ((st = upload_single(c, ws, s, hv.on ? &ex : nullptr)) != KPM_OK) return st;
  if (hv.on) {
    if ((st = run_forward_split(c, hv, false, mu, s)) != KPM_OK) return st;
  } else {
    if ((st = run_forward(c, false, M, s)) != KPM_OK) return st;
    if ((st = run_moments(c, mu, s)) != KPM_OK) return st;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_fwd.erase(ws);
  return KPM_OK;
}

int kpm_moments_noalloc(const kpm_lattice* lat, const double* h, const double* ab,
                        const kpm_probes* probes, int32_t M, int32_t precision, double* mu,
                        void* stream) {
  if (!mu || !valid_lattice(lat) || M < 2) return KPM_EINVAL;
  if (precision != KPM_FP64 && precision != KPM_FP32) return KPM_EINVAL;
  const int R = build_groups(lat, probes, nullptr, nullptr);
  if (R < 1 || !records_fit(lat, R)) return KPM_EINVAL;
  // forward-only layout (no gamma vectors, checkpoints or adjoint sums)
  const WsLayout w = ws_layout(sizes(lat, R, M, M, precision == KPM_FP32, true));
  if (w.total > (size_t)KPM_NOALLOC_SCRATCH_BYTES) return KPM_ETOOBIG;
  void* ws = nullptr;
  int st = scratch_address(&ws);
  if (st != KPM_OK) return st;
  Ctx c;
  st = prepare_single(c, lat, h, ab, probes, M, nullptr, precision, std::max<int32_t>(M, 2), ws,
                      KPM_NOALLOC_SCRATCH_BYTES, true);
  if (st != KPM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int tiles_x = (lat->Lx + kTX - 1) / kTX;
  const int nt = std::max(c.nch(), c.ntl());
  hipLaunchKernelGGL(k_fill_tables, dim3((nt + 255) / 256), dim3(256), 0, s, c.inst[0], c.d_inst,
                     c.d_cmap, c.d_tmap, c.nch(), c.ntl(), tiles_x);
  KPM_HIP(hipGetLastError());
  if ((st = run_forward(c, false, M, s)) != KPM_OK) return st;
  if ((st = run_moments(c, mu, s)) != KPM_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  g_fwd.erase(ws);
  return KPM_OK;
}

int kpm_grand_potential(const kpm_lattice* lat, const double* h, const double* ab,
                        const kpm_probes* probes, int32_t M, const double* C, int32_t precision,
                        int32_t ckpt_k, double* omega, double* mu, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!C || !omega) return KPM_EINVAL;
  Ctx c;
  int st = prepare_single(c, lat, h, ab, probes, M, C, precision, ckpt_k, ws, ws_bytes);
  if (st != KPM_OK) return st;
  c.inst[0].omega = omega;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Halves hv;
  if (split_wanted(c, s) && (st = setup_halves(c, hv, ws, s, true)) != KPM_OK) return st;
  if (hv.on) {
    const std::vector<InstDev> ex = hv.inst();
    if ((st = upload_single(c, ws, s, &ex)) != KPM_OK) return st;
    if ((st = run_forward_split(c, hv, true, mu, s)) != KPM_OK) return st;
  } else {
    if ((st = upload_single(c, ws, s)) != KPM_OK) return st;
    if ((st = tune_single(c, ws, s)) != KPM_OK) return st;
    if ((st = run_forward(c, true, M, s)) != KPM_OK) return st;
    if ((st = run_moments(c, mu, s)) != KPM_OK) return st;
  }
  KPM_HIP(launch_omega(c.d_inst, 1, M, s));
  std::lock_guard<std::mutex> lk(g_mu);
  g_fwd[ws] = FwdSig{h, ab, C, M, c.Rmax, precision, ckpt_k, false, hv.on};
  return KPM_OK;
}

int kpm_grand_potential_grad(const kpm_lattice* lat, const double* h, const double* ab,
                             const kpm_probes* probes, int32_t M, const double* C,
                             int32_t precision, int32_t ckpt_k, const double* omega_bar,
                             double* rho, void* ws, size_t ws_bytes, void* stream) {
  if (!C || !rho) return KPM_EINVAL;
  Ctx c;
  int st = prepare_single(c, lat, h, ab, probes, M, C, precision, ckpt_k, ws, ws_bytes);
  if (st != KPM_OK) return st;
  bool consumed, split;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_fwd.find(ws);
    if (it == g_fwd.end()) return KPM_EWORKSPACE;
    const FwdSig& f = it->second;
    if (f.h != h || f.ab != ab || f.C != C || f.M != M || f.R != c.Rmax || f.prec != precision ||
        f.k != ckpt_k)
      return KPM_EWORKSPACE;
    consumed = f.consumed;
    split = f.split;
  }
  c.inst[0].rho = reinterpret_cast<double2*>(rho);
  c.inst[0].omega_bar = omega_bar;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the adjoint follows the forward's layout: probe halves if it ran as halves
  Halves hv;
  if (split) {
    if ((st = setup_halves(c, hv, ws, s, false)) != KPM_OK) return st;
    if (!hv.on) return KPM_EWORKSPACE;
    const std::vector<InstDev> ex = hv.inst();
    if ((st = upload_single(c, ws, s, &ex)) != KPM_OK) return st;
    // a second adjoint after one forward (e.g. two backward passes): the first
    // one left alpha_0, alpha_1 in the ping-pong buffers
    if (consumed && (st = restore_alpha_split(hv, s)) != KPM_OK) return st;
    if ((st = run_adjoint_split(c, hv, s)) != KPM_OK) return st;
  } else {
    if ((st = upload_single(c, ws, s)) != KPM_OK) return st;
    if (consumed && (st = restore_alpha(c, s)) != KPM_OK) return st;
    if ((st = run_adjoint(c, s)) != KPM_OK) return st;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_fwd.find(ws);
  if (it != g_fwd.end()) it->second.consumed = true;
  return KPM_OK;
}

int kpm_density_matrix(const kpm_lattice* lat, const double* h, const double* ab,
                       const kpm_probes* probes, int32_t M, const double* C, int32_t precision,
                       int32_t ckpt_k, double* omega, double* rho, double* n_up, double* n_dn,
                       double* chi_up, double* chi_dn, double* delta_up, double* delta_dn,
                       void* ws, size_t ws_bytes, void* stream) {
  int st = kpm_grand_potential(lat, h, ab, probes, M, C, precision, ckpt_k, omega, nullptr, ws,
                               ws_bytes, stream);
  if (st != KPM_OK) return st;
  st = kpm_grand_potential_grad(lat, h, ab, probes, M, C, precision, ckpt_k, nullptr, rho, ws,
                                ws_bytes, stream);
  if (st != KPM_OK) return st;
  KPM_HIP(launch_map(lat->Lx * lat->Ly, rho, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn,
                     static_cast<hipStream_t>(stream)));
  return KPM_OK;
}

int kpm_density_matrix_direct(const kpm_lattice* lat, const double* h, const double* ab,
                              const kpm_probes* probes, int32_t M, const double* C,
                              int32_t precision, double* omega, double* rho, void* ws,
                              size_t ws_bytes, void* stream) {
  if (!C || !omega || !rho) return KPM_EINVAL;
  Ctx c;
  // no checkpoints are read: the smallest checkpoint area (interval M) suffices
  int st = prepare_single(c, lat, h, ab, probes, M, C, precision, std::max<int32_t>(M, 2), ws,
                          ws_bytes);
  if (st != KPM_OK) return st;
  c.inst[0].omega = omega;
  c.inst[0].rho = reinterpret_cast<double2*>(rho);
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_fwd.erase(ws);                       // the adjoint buffers are overwritten below
  }
  if ((st = upload_single(c, ws, s)) != KPM_OK) return st;
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, s, c.d_inst, 1, 0);
  KPM_HIP(hipGetLastError());
  KPM_HIP(launch_rescale(c.d_inst, c.d_tmap, c.ntl(), c.fp32, s));
  KPM_HIP(launch_direct_coef(c.d_inst, 1, M, s));
  KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, 0, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), 0, M, c.k, 0, c.bal, s));
  // step m writes alpha_{m+1}; even steps also add D_m alpha_m + D_{m+1} alpha_{m+1} to y
  for (int m = 0; m + 1 < M; ++m)
    KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, (m & 1) ? 1 : 5, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), m, M,
                        c.k, m == 0 ? 1 : 0, c.bal, s));
  if ((st = run_moments(c, nullptr, s)) != KPM_OK) return st;
  KPM_HIP(launch_omega(c.d_inst, 1, M, s));
  KPM_HIP(launch_rho_direct(c.d_inst, c.d_cmap, c.nch(), s));
  return KPM_OK;
}

int kpm_moments_doubling(const kpm_lattice* lat, const double* h, const double* ab,
                         const kpm_probes* probes, int32_t M, const double* C, int32_t precision,
                         double* omega, double* mu, void* ws, size_t ws_bytes, void* stream) {
  if ((C == nullptr) != (omega == nullptr) || (!mu && !omega)) return KPM_EINVAL;
  Ctx c;
  int st = prepare_single(c, lat, h, ab, probes, M, C, precision, std::max<int32_t>(M, 2), ws,
                          ws_bytes);
  if (st != KPM_OK) return st;
  c.inst[0].omega = omega;
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_fwd.erase(ws);
  }
  if ((st = upload_single(c, ws, s)) != KPM_OK) return st;
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, s, c.d_inst, 1, 0);
  KPM_HIP(hipGetLastError());
  KPM_HIP(launch_rescale(c.d_inst, c.d_tmap, c.ntl(), c.fp32, s));
  KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, 0, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), 0, M, c.k, 0, c.bal, s));
  // alpha_1 .. alpha_{M/2}: every moment slot below M is then written
  for (int m = 0; m < M / 2; ++m)
    KPM_HIP(launch_cheb(c.fp32, c.Pf, c.Sf, 4, c.d_inst, c.d_tmap, c.ntl(), c.tpx(), c.nrf(), m, M, c.k, 0, c.bal, s));
  if ((st = run_moments(c, nullptr, s)) != KPM_OK) return st;
  KPM_HIP(launch_mom_double(c.d_inst, 1, c.inst[0].R * M, M, mu, s));
  if (omega) KPM_HIP(launch_omega(c.d_inst, 1, M, s));
  return KPM_OK;
}

int kpm_ldos(const kpm_lattice* lat, const double* h, const double* ab, int32_t first,
             int32_t count, int32_t M, int32_t precision, const double* energies, int32_t ne,
             double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!energies || !out || ne < 1 || count < 1 || count > 65535 || first < 0) return KPM_EINVAL;
  kpm_probe_group g{};
  g.kind = KPM_PROBE_UNIT;
  g.count = count;
  g.first = first;
  g.px = g.py = 1;
  g.weight = 1.0;
  const kpm_probes pr{&g, 1};
  Ctx c;
  int st = prepare_single(c, lat, h, ab, &pr, M, nullptr, precision, std::max<int32_t>(M, 2), ws,
                          ws_bytes);
  if (st != KPM_OK) return st;
  if ((long long)ne * count >= (1LL << 31)) return KPM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_fwd.erase(ws);
  }
  if ((st = upload_single(c, ws, s)) != KPM_OK) return st;
  if ((st = run_forward(c, false, M, s)) != KPM_OK) return st;
  if ((st = run_moments(c, nullptr, s)) != KPM_OK) return st;
  KPM_HIP(launch_ldos(c.d_inst, count, M, energies, ne, out, s));
  return KPM_OK;
}

int kpm_status_read(const void* ws, int32_t* status, void* stream) {
  if (!ws || !status) return KPM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the status word is the first field of the instance buffers
  InstDev I;
  KPM_HIP(hipMemcpyAsync(&I, ws, sizeof(InstDev), hipMemcpyDeviceToHost, s));
  KPM_HIP(hipStreamSynchronize(s));
  int v = 0;
  if (I.status) {
    KPM_HIP(hipMemcpyAsync(&v, I.status, sizeof(int), hipMemcpyDeviceToHost, s));
    KPM_HIP(hipStreamSynchronize(s));
  }
  *status = v;
  return KPM_OK;
}

int32_t kpm_set_probe_block(int32_t probes_per_thread) {
  std::lock_guard<std::mutex> lk(g_mu);
  int32_t old = g_probe_block;
  if (probes_per_thread == 0 || valid_P(probes_per_thread)) g_probe_block = probes_per_thread;
  return old;
}

int32_t kpm_set_streams(int32_t n) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int32_t old = g_streams;
  if (n >= 0 && n <= 2) g_streams = n;
  return old;
}

int kpm_set_schedule(int32_t fwd, int32_t adj) {
  auto ok = [](int32_t v) { return v >= KPM_SCHED_DEFAULT && v <= KPM_SCHED_BALANCED; };
  if (!ok(fwd) || !ok(adj)) return KPM_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  g_sched_f = fwd;
  g_sched_a = adj;
  return KPM_OK;
}

int kpm_batch_tuning(const void* plan, int32_t* out) {
  if (!plan || !out) return KPM_EINVAL;
  const KpmBatchPlan* pl = static_cast<const KpmBatchPlan*>(plan);
  if (!pl->groups.empty()) pl = pl->groups[0];
  const Ctx& c = pl->hv.on ? pl->hv.h[0] : pl->c;
  out[0] = c.Pf;
  out[1] = c.Sf;
  out[2] = c.Pa;
  out[3] = c.Sa;
  out[4] = pl->tune_source;
  return KPM_OK;
}

int32_t kpm_batch_streams(const void* plan) {
  if (!plan) return KPM_EINVAL;
  const auto* pl = static_cast<const KpmBatchPlan*>(plan);
  int32_t n = pl->hv.on ? 2 : 1;
  for (const KpmBatchPlan* g : pl->groups) n = std::max(n, (int32_t)(g->hv.on ? 2 : 1));
  return n;
}

}  // extern "C"

namespace {

// A plan over all of the given instances (no groups).
int batch_create_leaf(int32_t n_inst, const kpm_lattice* lats, const kpm_probes* probes, int32_t M,
                      int32_t precision, int32_t ckpt_k, KpmBatchPlan** plan) {
  const bool fp32 = precision == KPM_FP32;
  std::vector<Sizes> zs(n_inst);
  std::vector<InstDev> insts(n_inst);
  size_t total = align_up(sizeof(InstDev) * n_inst);
  size_t nch = 0, ntl = 0;
  for (int q = 0; q < n_inst; ++q) {
    if (!valid_lattice(&lats[q])) return KPM_EINVAL;
    std::memset(&insts[q], 0, sizeof(InstDev));
    int ng = 0;
    const int R = build_groups(&lats[q], &probes[q], insts[q].g, &ng);
    if (R < 1 || !records_fit(&lats[q], R)) return KPM_EINVAL;
    zs[q] = sizes(&lats[q], R, M, ckpt_k, fp32);
    insts[q].Lx = lats[q].Lx;
    insts[q].Ly = lats[q].Ly;
    insts[q].N = zs[q].N;
    insts[q].R = R;
    insts[q].nchunk = zs[q].ntile;
    insts[q].ngroups = ng;
    nch += zs[q].nchunk;
    ntl += zs[q].ntile;
    total += inst_bytes(zs[q]);
  }
  total += align_up(sizeof(int2) * nch) + align_up(sizeof(int4) * ntl);
  const bool split = batch_split_wanted(insts);
  // the halves' tables: n_inst entries, nch chunks and ntl tiles between them
  // (each table aligned on its own)
  const size_t half_tables = split ? 2 * (align_up(sizeof(InstDev) * n_inst) + align_up(sizeof(int2) * nch) +
                                          align_up(sizeof(int4) * ntl))
                                   : 0;
  total += half_tables;
  auto* pl = new (std::nothrow) KpmBatchPlan();
  if (!pl) return KPM_ENOMEM;
  if (hipMalloc(&pl->mem, total) != hipSuccess) {
    delete pl;
    return KPM_ENOMEM;
  }
  char* base = static_cast<char*>(pl->mem);
  pl->c.d_inst = reinterpret_cast<InstDev*>(base);
  char* o = base + align_up(sizeof(InstDev) * n_inst);
  pl->c.d_cmap = reinterpret_cast<int2*>(o);
  o += align_up(sizeof(int2) * nch);
  pl->c.d_tmap = reinterpret_cast<int4*>(o);
  o += align_up(sizeof(int4) * ntl);
  for (int q = 0; q < n_inst; ++q) {
    carve(insts[q], zs[q], o);
    o += inst_bytes(zs[q]);
  }
  pl->c.inst = insts;
  pl->c.M = M;
  pl->c.k = ckpt_k;
  pl->c.fp32 = fp32;
  finish_ctx(pl->c);
  int P;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    P = g_probe_block;
    pl->c.Sf = g_sched_f;
    pl->c.Sa = g_sched_a;
  }
  pl->c.Pf = P ? P : auto_probe_fwd(pl->c.ntl(), pl->c.Rmax);
  pl->c.Pa = P ? P : auto_probe_adj(pl->c.ntl(), pl->c.Rmax);
  pl->tuned = P != 0;
  set_npb(pl->c);
  if (split) {
    split_instances(insts, pl->idx);
    for (int q = 0; q < 2; ++q) {
      Ctx& h = pl->hv.h[q];
      h.inst.clear();
      for (int j : pl->idx[q]) h.inst.push_back(pl->c.inst[j]);
      h.M = M;
      h.k = ckpt_k;
      h.fp32 = fp32;
      h.Sf = pl->c.Sf;
      h.Sa = pl->c.Sa;
      finish_ctx(h);
      h.d_inst = reinterpret_cast<InstDev*>(o);
      o += align_up(sizeof(InstDev) * h.inst.size());
      h.d_cmap = reinterpret_cast<int2*>(o);
      o += align_up(sizeof(int2) * h.cmap.size());
      h.d_tmap = reinterpret_cast<int4*>(o);
      o += align_up(sizeof(int4) * h.tmap.size());
      h.Pf = P ? P : auto_probe_fwd(h.ntl(), h.Rmax);
      h.Pa = P ? P : auto_probe_adj(h.ntl(), h.Rmax);
      set_npb(h);
    }
    npb_from_halves(pl);
    pl->hv.on = true;
  }
  *plan = pl;
  return KPM_OK;
}

// Energy + gradient of a plan without groups; omega: one device pointer per instance.
int batch_run_leaf(KpmBatchPlan* pl, const double* const* h, const double* const* ab,
                   const double* const* C, double* const* omega, double* const* rho, int32_t use_graph,
                   hipStream_t s) {
  Ctx& c = pl->c;
  const int n = (int)c.inst.size();
  std::vector<const void*> ptrs;
  for (int q = 0; q < n; ++q) {
    if (!h[q] || !ab[q] || !C[q] || !rho[q]) return KPM_EINVAL;
    c.inst[q].h = reinterpret_cast<const double2*>(h[q]);
    c.inst[q].ab = ab[q];
    c.inst[q].C = C[q];
    c.inst[q].omega = omega[q];
    c.inst[q].rho = reinterpret_cast<double2*>(rho[q]);
    c.inst[q].omega_bar = nullptr;
    ptrs.insert(ptrs.end(), {h[q], ab[q], C[q], omega[q], rho[q]});
  }
  int st;
  if (!pl->tuned) {
    if (pl->hv.on) {
      // both halves take one pick, timed on the pair
      auto prep = [&](const Tune& t) -> int {
        for (int q = 0; q < 2; ++q) apply_tune(pl->hv.h[q], t);
        npb_from_halves(pl);
        return upload_plan(pl, s);
      };
      if ((st = upload_plan(pl, s)) != KPM_OK) return st;
      if ((st = tune_pair(c, pl->hv, shape_key(c) + "/2", prep, s, true, &pl->tune_source)) != KPM_OK)
        return st;
    } else {
      if ((st = upload(c, s)) != KPM_OK) return st;
      if ((st = tune_ctx(pl->c, nullptr, s, &pl->tune_source)) != KPM_OK) return st;
    }
    pl->tuned = true;
  }
  if ((st = upload_plan(pl, s)) != KPM_OK) return st;
  if (!use_graph) return batch_sequence(pl, s);
  if (pl->exec && pl->graph_ptrs != ptrs) {
    (void)hipGraphExecDestroy(pl->exec);
    (void)hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
    if (pl->exec2) (void)hipGraphExecDestroy(pl->exec2);
    if (pl->graph2) (void)hipGraphDestroy(pl->graph2);
    pl->exec2 = nullptr;
    pl->graph2 = nullptr;
  }
  if (!pl->exec) {
    // The captured kernels read the instance tables from device memory, so a
    // graph stays valid as long as the tables are re-uploaded before each
    // replay.  Capture on private streams (the caller's may be the null
    // stream, which cannot be captured); nothing runs during capture.  With
    // instance halves each half is captured whole (its own status words,
    // moments, Omega and rho) as a graph of its own, and the two graphs are
    // launched on the two streams.
    auto capture = [](hipStream_t& cs, Ctx& cc, hipGraph_t& graph, hipGraphExec_t& exec) -> int {
      if (!cs) KPM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      KPM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      const int r = batch_sequence_ctx(cc, cs);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &g);
      if (r != KPM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return r != KPM_OK ? r : KPM_EDEVICE;
      }
      if (hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        exec = nullptr;
        return KPM_EDEVICE;
      }
      graph = g;
      return KPM_OK;
    };
    if (pl->hv.on) {
      if ((st = capture(pl->capture_stream, pl->hv.h[0], pl->graph, pl->exec)) != KPM_OK) return st;
      if ((st = capture(pl->capture2, pl->hv.h[1], pl->graph2, pl->exec2)) != KPM_OK) {
        // capture again on the next call
        if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
        if (pl->graph) (void)hipGraphDestroy(pl->graph);
        pl->exec = nullptr;
        pl->graph = nullptr;
        return st;
      }
    } else if ((st = capture(pl->capture_stream, pl->c, pl->graph, pl->exec)) != KPM_OK) {
      return st;
    }
    pl->graph_ptrs = ptrs;
  }
  if (!pl->hv.on) {
    KPM_HIP(hipGraphLaunch(pl->exec, s));
    return KPM_OK;
  }
  Fork f;
  if ((st = fork_from(f, s)) != KPM_OK) return st;
  KPM_HIP(hipGraphLaunch(pl->exec, s));
  KPM_HIP(hipGraphLaunch(pl->exec2, f.s2));
  return join_to(f, s);
}

void batch_destroy_plan(KpmBatchPlan* pl) {
  for (KpmBatchPlan* g : pl->groups) batch_destroy_plan(g);
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->exec2) (void)hipGraphExecDestroy(pl->exec2);
  if (pl->graph2) (void)hipGraphDestroy(pl->graph2);
  if (pl->capture_stream) (void)hipStreamDestroy(pl->capture_stream);
  if (pl->capture2) (void)hipStreamDestroy(pl->capture2);
  if (pl->mem) {
    (void)hipDeviceSynchronize();
    (void)hipFree(pl->mem);
  }
  delete pl;
}

}  // namespace

extern "C" {

int kpm_batch_create(int32_t n_inst, const kpm_lattice* lats, const kpm_probes* probes, int32_t M,
                     int32_t precision, int32_t ckpt_k, void** plan) {
  if (n_inst < 1 || !lats || !probes || !plan || M < 2 || ckpt_k < 2) return KPM_EINVAL;
  if (precision != KPM_FP64 && precision != KPM_FP32) return KPM_EINVAL;
  std::vector<long long> rn(n_inst);
  for (int q = 0; q < n_inst; ++q) {
    if (!valid_lattice(&lats[q])) return KPM_EINVAL;
    const int R = build_groups(&lats[q], &probes[q], nullptr, nullptr);
    if (R < 1 || !records_fit(&lats[q], R)) return KPM_EINVAL;
    rn[q] = (long long)R * lats[q].Lx * lats[q].Ly;
  }
  const int G = batch_group_count(rn, precision == KPM_FP32);
  KpmBatchPlan* pl = nullptr;
  if (G <= 1) {
    const int st = batch_create_leaf(n_inst, lats, probes, M, precision, ckpt_k, &pl);
    if (st != KPM_OK) return st;
    *plan = pl;
    return KPM_OK;
  }
  pl = new (std::nothrow) KpmBatchPlan();
  if (!pl) return KPM_ENOMEM;
  pl->gidx = group_instances(rn, G);
  for (const auto& idx : pl->gidx) {
    std::vector<kpm_lattice> gl;
    std::vector<kpm_probes> gp;
    for (int q : idx) {
      gl.push_back(lats[q]);
      gp.push_back(probes[q]);
    }
    KpmBatchPlan* leaf = nullptr;
    const int st = batch_create_leaf((int32_t)idx.size(), gl.data(), gp.data(), M, precision, ckpt_k, &leaf);
    if (st != KPM_OK) {
      batch_destroy_plan(pl);
      return st;
    }
    pl->groups.push_back(leaf);
  }
  *plan = pl;
  return KPM_OK;
}

int kpm_batch_energy_grad(void* plan, const double* const* h, const double* const* ab,
                          const double* const* C, double* omega, double* const* rho,
                          int32_t use_graph, void* stream) {
  auto* pl = static_cast<KpmBatchPlan*>(plan);
  if (!pl || !h || !ab || !C || !omega || !rho) return KPM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->groups.empty()) {
    std::vector<double*> om(pl->c.inst.size());
    for (size_t q = 0; q < om.size(); ++q) om[q] = omega + q;
    return batch_run_leaf(pl, h, ab, C, om.data(), rho, use_graph, s);
  }
  for (size_t g = 0; g < pl->groups.size(); ++g) {
    const auto& idx = pl->gidx[g];
    std::vector<const double*> gh, gab, gC;
    std::vector<double*> gom, grho;
    for (int q : idx) {
      gh.push_back(h[q]);
      gab.push_back(ab[q]);
      gC.push_back(C[q]);
      gom.push_back(omega + q);
      grho.push_back(rho[q]);
    }
    const int st = batch_run_leaf(pl->groups[g], gh.data(), gab.data(), gC.data(), gom.data(), grho.data(),
                                  use_graph, s);
    if (st != KPM_OK) return st;
  }
  return KPM_OK;
}

int32_t kpm_batch_groups(const void* plan) {
  if (!plan) return KPM_EINVAL;
  const auto* pl = static_cast<const KpmBatchPlan*>(plan);
  return pl->groups.empty() ? 1 : (int32_t)pl->groups.size();
}

int32_t kpm_set_batch_groups(int32_t groups) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int32_t old = g_batch_groups;
  if (groups >= 0) g_batch_groups = groups;
  return old;
}

int kpm_batch_destroy(void* plan) {
  auto* pl = static_cast<KpmBatchPlan*>(plan);
  if (!pl) return KPM_EINVAL;
  batch_destroy_plan(pl);
  return KPM_OK;
}

int kpm_profile_begin(int32_t sample_every) {
  if (sample_every < 1) return KPM_EINVAL;
  KPM_HIP(profile_begin(sample_every));
  return KPM_OK;
}

int kpm_profile_end(double* fwd_ms, int32_t* n_fwd, double* adj_ms, int32_t* n_adj) {
  if (!fwd_ms || !n_fwd || !adj_ms || !n_adj) return KPM_EINVAL;
  int nf = 0, na = 0;
  KPM_HIP(profile_end(fwd_ms, &nf, adj_ms, &na));
  *n_fwd = nf;
  *n_adj = na;
  return KPM_OK;
}

const char* kpm_strerror(int status) {
  switch (status) {
    case KPM_OK: return "ok";
    case KPM_EINVAL: return "invalid argument";
    case KPM_ENOMEM: return "out of device memory";
    case KPM_EDEVICE: return "HIP runtime error";
    case KPM_EBOUNDS: return "spectrum outside the rescaled interval or non-finite value";
    case KPM_ENOTSUP: return "not supported";
    case KPM_EWORKSPACE: return "workspace too small or not prepared by the forward call";
    case KPM_ENOCONV: return "chemical-potential search used its evaluation budget";
    case KPM_ETOOBIG: return "problem larger than the library's static scratch (KPM_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

}  // extern "C"
