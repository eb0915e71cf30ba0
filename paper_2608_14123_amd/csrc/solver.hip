// Host orchestration: level hierarchy and geometry set-up, WAS (Alg. 5), SCG
// (Alg. 6), the FAS V-cycle (Alg. 2) and the C ABI of include/dgfas.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dgfas.h"
#include "blas.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "tables.hpp"
#include "mlp.hpp"
#include "topology.hpp"

namespace dgfas {
namespace {

thread_local std::string g_err;

struct Error : std::runtime_error {
  dgfas_status code;
  Error(dgfas_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPC(x)                                                                                   \
  do {                                                                                            \
    hipError_t e_ = (x);                                                                          \
    if (e_ != hipSuccess)                                                                         \
      throw Error(DGFAS_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));                    \
  } while (0)


// Overlap inbox of dgfas_schwarz_noalloc.  Every device holds its own copy of the array; its
// address on each device is resolved once (hipGetSymbolAddress, with that device current) at
// the first solver creation there, and host code uses only the resolved address.
constexpr size_t kNoAllocDoubles = (size_t)8 << 20;   // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// resolve the array's address on the current device (called at set-up)
void resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(DGFAS_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw Error(DGFAS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = static_cast<double*>(ptr);
}

double* scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

template <typename T>
T* dalloc(size_t n) {
  if (n == 0) return nullptr;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw Error(DGFAS_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  return static_cast<T*>(p);
}

template <typename T>
T* upload(const std::vector<T>& h, hipStream_t st) {
  T* d = dalloc<T>(h.size());
  if (d) HIPC(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return d;
}

template <typename T>
std::vector<T> download(const T* d, size_t n, hipStream_t st) {
  std::vector<T> h(n);
  if (n) HIPC(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return h;
}

std::vector<float> to_float(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

// Tables of one polynomial degree, shared by every level holding elements of that degree:
// GLL data, the differentiation matrix and the 16 Schwarz variants (side codes I, D, N, I0
// per direction end, zero padded to ns = p + 1 + 2m).
struct DegTab {
  int p = 0, n = 0, m = 0, ns = 0;
  double inv_wend = 0;
  double *D = nullptr, *w1 = nullptr, *x1 = nullptr;
  float* D32 = nullptr;
  double *S = nullptr, *ST = nullptr, *lam = nullptr, *W = nullptr;
  float *S32 = nullptr, *ST32 = nullptr, *lam32 = nullptr, *W32 = nullptr;
  int* map1d = nullptr;
  std::vector<double> h_W;   // host copies of the weights and node maps [16][ns]
  std::vector<int> h_map;
};

// The elements of one degree on a level (the whole level when it is uniform, elist = null),
// with the transfer matrices to the next coarser level.
struct Bucket {
  int p = 0, n = 0, nel = 0;
  int* elist = nullptr;
  std::vector<int> h_elist;
  DegTab* t = nullptr;
  int pc = 0;                                        // coarse degree of these elements
  double *Pm = nullptr, *Im = nullptr, *Rm = nullptr;
};

// element classes of local refinement (Sec. 3.1)
const int8_t kTwig = 0, kLeaf = 1, kFrozen = 2;
const int8_t kLevelEdge = 3;   // host only: a frozen element's face toward the unrefined region

struct Level {
  int p = 0, n = 0, N2 = 0, N3 = 0, E = 0, m = 0, ns = 0;   // p: largest degree on the level
  bool uniform = true;
  // topology of this level (a level below an h-coarsening has an eighth of the elements)
  int* nbr = nullptr;
  int8_t* bc = nullptr;
  std::vector<int> h_nbr;
  std::vector<int8_t> h_bc;
  int box[3] = {0, 0, 0};
  // the next coarser level is this one h-coarsened (Sec. 3.1): parents of 2 x 2 x 2 children
  bool hdown = false;
  int* hchild = nullptr;                // [E of the coarser level][8] children of every parent
  double* hM = nullptr;                 // [6][n][n] P_0, P_1, I_0^T, I_1^T, I_0, I_1
  // local refinement (Sec. 3.1): element classes; the sweep kernels run over the active
  // elements, frozen ones are data.  The transfer lists to the level below sit on the finer
  // level: twig parents with their active children, irregular (leaf) parents with their frozen
  // children.
  bool lr = false;
  std::vector<int8_t> h_cls;            // kTwig / kLeaf / kFrozen per element
  int nact = 0, nleaf = 0, ntwig = 0;
  int *act_list = nullptr, *leaf_list = nullptr, *twig_list = nullptr;
  int* sdeg = nullptr;                  // degree per element for the Schwarz kernels, frozen -1
  bool lr_down = false;                 // built from the level below by local refinement
  int ntw = 0, nir = 0;
  int *tw_par = nullptr, *tw_ch = nullptr, *ir_par = nullptr, *ir_ch = nullptr;
  double* sq = nullptr;                 // [nleaf] composite-residual partials
  double* bfull = nullptr;              // the level's discrete right-hand side (levels below the
                                        // top; library memory, kept between calls)
  int64_t ndof = 0, nfs = 0, nin = 0;   // nodes, face-node slots and inbox slots per right-hand side
  double inv_wend = 0;
  std::vector<int> h_deg;
  std::vector<int64_t> h_off;
  int* deg = nullptr;                   // device per-element data, null on uniform levels
  int64_t *off = nullptr, *offF = nullptr, *offO = nullptr;
  std::vector<Bucket> bk;
  // one-launch batches over the buckets (levels with several degrees)
  BucketDesc<double>* bd64 = nullptr;
  BucketDesc<float>* bd32 = nullptr;
  int tiles[3] = {0, 0, 0};             // work-list length per stage
  int one_launch[3] = {0, 0, 0};        // tuned choice per stage: 0 per degree, 1 one launch,
                                        // 2 one persistent launch
  std::string hist;                     // degree histogram "p:count,..." (autotuner key)
  bool all_m1 = true;                   // every degree bucket has overlap 1 (batched Schwarz tiles)
  int nm = 0;                           // elements with a face to another degree
  int nlb = 0;                          // operator tiles per right-hand side (uniform levels)
  double* kpart = nullptr;              // [nrhs][nlb] fused p^T A p partial sums (uniform levels)
  int nla = 0;                          // overlap-add tiles per right-hand side (uniform levels)
  double* zpart = nullptr;              // [2][nrhs][nla] fused z^T r, z^T (r - r0) partial sums
  int nmf = 0;                          // faces to another degree (one task per face)
  int64_t* mfdesc = nullptr;            // [nmf][8] face descriptors (MortarArgs::fdesc)
  int* mfmapE = nullptr;                // [E][6] result slot of face phi, or -1
  double* mfres = nullptr;              // [nrhs][2 nmf][4][81] face results per side
  double* muf = nullptr;                // [E][6] mu_F nu
  // geometry
  double *X = nullptr, *G = nullptr, *WJ = nullptr, *ws = nullptr, *pen = nullptr;
  double *vol = nullptr, *area = nullptr, *lin = nullptr;
  double* nun = nullptr;         // nodal diffusivity of the level, or null (the scalar nu)
  double* nuavg = nullptr;       // [E] element averages of nun
  float *G32 = nullptr, *WJ32 = nullptr, *pen32 = nullptr;
  // Schwarz
  int* nb27 = nullptr;
  int8_t* var = nullptr;
  double *gco = nullptr, *O = nullptr;
  float *gco32 = nullptr, *O32 = nullptr;
  double* cinv = nullptr;        // [ndof] 1 / weight sum per node where the tensor weights of the
  float* cinv32 = nullptr;       // subdomains reaching it do not add up to one; null on uniform levels
  double* J9 = nullptr;          // [E][9] linear map Jacobian / det^(1/3) (network input)
  // unstructured mesh (the neighbours' faces and orientations of Sec. 5.1): the operator reads
  // its neighbours through nfo, the Schwarz method runs from the slot tables of topology.cpp
  bool topo = false;
  int8_t* nfo = nullptr;         // [E][6] the neighbour's face | orientation << 3
  std::vector<int8_t> h_nface, h_norient;
  int tnt = 0;                   // slots per tile
  int *tg = nullptr, *tmptr = nullptr, *tmidx = nullptr, *tsslot = nullptr;
  int64_t* tsptr = nullptr;
  double* tscoef = nullptr;
  float* tscoef32 = nullptr;
  double* Zt = nullptr;          // [nrhs][E][tnt] subdomain solutions (workspace)
  float* Zt32 = nullptr;
  int64_t tblocks[5] = {0, 0, 0, 0, 0};
  std::vector<int> h_nb27;       // host copy of the 26-neighbourhood
  // vectors
  double *u = nullptr, *g = nullptr, *ubar = nullptr, *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr,
         *r0 = nullptr;
  float *r32 = nullptr, *du32 = nullptr, *rc32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr,
        *r0_32 = nullptr;
  // after an FP64 SCG smoothing call: the buffer holding its recurrence residual g - A u of
  // the smoothed u (r or r0, by the parity of the iteration count); null otherwise
  const double* rsm = nullptr;

  template <typename T>
  void scg_vectors(T*& r_, T*& z_, T*& p_, T*& q_, T*& r0_) {
    if constexpr (sizeof(T) == 8) { r_ = r; z_ = z; p_ = pv; q_ = q; r0_ = r0; }
    else { r_ = rc32; z_ = z32; p_ = p32; q_ = q32; r0_ = r0_32; }
  }
};

struct Solver {
  dgfas_options opt{};
  hipStream_t st = nullptr;
  int E = 0;
  int* nbr = nullptr;
  int8_t* bc = nullptr;
  std::vector<int> h_nbr;
  std::vector<int8_t> h_bc;
  std::vector<Level> lv;   // lv[0] = root (level 1)
  std::vector<int64_t> rank;   // processing rank of every element (empty: natural order)
  double* npart = nullptr;     // [nrhs][1024] block sums of the range projection (null_space)
  std::map<int, DegTab> tabs;
  double *Dall = nullptr, *Iall = nullptr;   // mixed-degree face tables for degrees 1..8
  int force_batch = -1;                      // autotuner: -1 options, 0 per degree, 1 one launch,
                                             // 2 one persistent launch
  int cus = 256;                             // compute units of the device
  // captured V-cycle legs (smoothing and transfers above the root, down and up)
  hipStream_t cap = nullptr;
  hipGraphExec_t gdown = nullptr, gup = nullptr;
  const double *gu = nullptr, *gf = nullptr;
  int graph_epoch = 0, graph_built_epoch = -1;
  // set by the solve loop right before a cycle: the finest level's r already holds g - A u for
  // the cycle's (u, g), so the first smoothing step need not recompute it (one-shot; cleared
  // once the cycle's pre-smoothing on the finest level has run)
  bool rhint = false;
  bool graph_hint = false;
  int ns1_top = -1;        // finest-level pre-smoothing steps of the next cycle (crossover); -1: ns1
  int graph_ns1 = -1;      // ns1_top the captured graphs were built with
  int nrhs = 1;            // right-hand sides per batch; vectors are [nrhs][ndof]
  int dev = 0;             // device the solver was created on
  double* inbox64 = nullptr;   // when set: FP64 overlap inbox of the Schwarz calls instead of L.O
  double* partial = nullptr;   // [2][nrhs][1024] first-stage sums
  double* scal = nullptr;      // [nrhs][8] SCG scalars
  double* partial2() { return partial + (size_t)1024 * nrhs; }
  double* dotout = nullptr;    // [nrhs] results of dots_sync
  std::vector<void*> owned;
  // learned correction on the finest level (FP64 Schwarz applications)
  Mlp* mlp = nullptr;
  bool learned = false;
  float *lX = nullptr, *lY = nullptr;
  double* lnorm = nullptr;
  double plain_rho = -1.0;       // first-cycle reduction factor of the plain smoother (fallback judge)
  double* usave = nullptr;       // finest-level copy of u taken before every learned cycle
  bool judge = true;             // apply the fallback rule (off only for diagnostics)
  // masked local solves (data generation): Schwarz restricted to selected subdomains, unweighted
  const uint8_t* msel = nullptr;
  const double* mmask = nullptr;

  template <typename T>
  T* own(T* p) {
    if (p) owned.push_back(p);
    return p;
  }
  // Workspace: the per-call scratch of the configured cycle (work vectors of every level,
  // overlap inboxes, reduction partials, SCG scalars).  Slots are registered during set-up and
  // laid out in one block, 256-byte aligned; the block is the library's own until
  // dgfas_set_workspace hands in a caller's buffer.  The slots carry no state between calls.
  struct WsSlot {
    void** p;
    size_t bytes;
    int zero;          // 0: none, 8 / 4: cleared as doubles / floats when assigned
  };
  std::vector<WsSlot> ws;
  void* ws_block = nullptr;   // library-owned block, null while a caller's buffer is in use
  size_t ws_bytes = 0;
  template <typename T>
  void reserve(T*& slot, size_t n, bool zero = false) {
    slot = nullptr;
    if (n) ws.push_back({reinterpret_cast<void**>(&slot), n * sizeof(T), zero ? (int)sizeof(T) : 0});
  }
  static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
  size_t ws_layout() const {
    size_t off = 0;
    for (const WsSlot& w : ws) off = align256(off) + w.bytes;
    return align256(off);
  }
  void ws_assign(char* base) {
    size_t off = 0;
    for (const WsSlot& w : ws) {
      off = align256(off);
      *w.p = base + off;
      if (w.zero == 8) fill((int64_t)(w.bytes / 8), static_cast<double*>(*w.p), 0.0, st);
      if (w.zero == 4) fill((int64_t)(w.bytes / 4), static_cast<float*>(*w.p), 0.0f, st);
      off += w.bytes;
    }
    for (Level& L : lv) L.rsm = nullptr;
    ++graph_epoch;   // captured graphs hold the old addresses
  }
  ~Solver() {
    if (st) hipStreamSynchronize(st);
    drop_graphs();
    if (cap) hipStreamDestroy(cap);
    for (void* p : owned) hipFree(p);
    if (ws_block) hipFree(ws_block);
  }
  void drop_graphs() {
    if (gdown) hipGraphExecDestroy(gdown);
    if (gup) hipGraphExecDestroy(gup);
    gdown = gup = nullptr;
    gu = gf = nullptr;
  }

  // one launch over all buckets for this level and stage?
  bool use_batch(const Level& L, int stage) const {
    if (L.uniform || L.bk.size() < 2) return false;
    if (stage != kStageOp && !L.all_m1) return false;   // batched Schwarz tiles take m = 1
    if (stage == kStageSolve && matrix_cores()) return false;   // matrix-core tiles per degree
    return batch_mode(L, stage) != 0;
  }
  int batch_mode(const Level& L, int stage) const {
    if (force_batch >= 0) return force_batch;
    if (opt.batch == DGFAS_BATCH_ONE_LAUNCH) return 1;
    if (opt.batch == DGFAS_BATCH_PERSISTENT) return 2;
    if (opt.batch == DGFAS_BATCH_TUNED) return L.one_launch[stage];
    return 0;
  }
  // workgroups of a one-launch batch: one per tile, or a persistent grid that strides through
  // the tiles (a multiple of 8, so that the round-robin XCD order of the tiles is kept)
  // A persistent launch keeps about 24 waves per CU: the workgroups per CU follow the stage's
  // workgroup width at the level's largest degree (2 for the 768-thread operator tile at p = 8,
  // 12 for the 2-wave subdomain solve, 6 for the 4-wave overlap add).
  int persistent_grid(int stage, int pmax) const {
    const int waves = std::max(1, stage_threads(stage, pmax) / 64);
    const int per_cu = std::max(1, 24 / waves);
    return 8 * std::max(1, (cus * per_cu + 7) / 8);
  }
  int batch_grid(const Level& L, int stage, int ntiles) const {
    if (batch_mode(L, stage) == 2) {
      const int g = persistent_grid(stage, L.p);
      if (ntiles > g) return g;
    }
    return xcd_grid(ntiles);
  }
  template <typename T>
  const BucketDesc<T>* bdesc(const Level& L) const {
    if constexpr (sizeof(T) == 8) return L.bd64;
    else return L.bd32;
  }

  Level& level(int l) {
    if (l < 1 || l > (int)lv.size()) throw Error(DGFAS_EINVAL, "level out of range");
    return lv[l - 1];
  }

  // ---------------------------------------------------------------- operator
  template <typename T>
  OpArgs<T> op_args(Level& L, const Bucket& b, int mode, const T* u, const T* g, T* out);

  // out = A u (mode 1) or g - A u (mode 0): the faces between degrees first, then one launch
  // per degree bucket (or one batched launch), which adds their terms
  template <typename T>
  void op(Level& L, int mode, const T* u, const T* g, T* out) {
    if (L.nm) {
      MortarArgs<T> m;
      m.nrhs = nrhs; m.ndof = L.ndof; m.u = u; m.ws = L.ws; m.muf = L.muf;
      m.Dall = Dall; m.Iall = Iall;
      m.nface = L.nmf; m.fdesc = L.mfdesc; m.fres = L.mfres;
      if constexpr (sizeof(T) == 8) m.G = L.G;
      else m.G = L.G32;
      sipg_mortar_faces<T>(m, st);
    }
    if (use_batch(L, kStageOp)) {
      OpArgs<T> a = op_args<T>(L, L.bk[0], mode, u, g, out);
      BatchLaunch bl;
      bl.nb = (int)L.bk.size(); bl.ntiles = L.tiles[kStageOp]; bl.grid = batch_grid(L, kStageOp, bl.ntiles); bl.persistent = bl.grid < bl.ntiles;
      sipg_apply_batched<T>(L.p, a, bdesc<T>(L), bl, st);
    } else {
      for (const Bucket& b : L.bk) {
        OpArgs<T> a = op_args<T>(L, b, mode, u, g, out);
        sipg_apply<T>(b.p, a, st);
      }
    }
  }
  void apply(Level& L, const double* u, double* Au) { op<double>(L, 1, u, nullptr, Au); }
  void residual(Level& L, const double* u, const double* g, double* r) { op<double>(L, 0, u, g, r); }
  void residual32(Level& L, const float* u, const float* g, float* r) { op<float>(L, 0, u, g, r); }

  template <typename T>
  SchwarzArgs<T> sz_args(Level& L, const Bucket& b, const T* r, T* z, int mode);

  // FD solve plus the network correction |r_s| MLP(r_s / |r_s|, J9) (finest level, FP64)
  void add_learned(Level& L, SchwarzArgs<double>& a, const double* r) {
    tile_features<double>(L.p, L.m, a, nullptr, L.E, r, L.J9, lX, lnorm, st);
    mlp->forward(lX, L.E, lY);
    a.corr = lY;
    a.cscale = lnorm;
  }
  void add_learned(Level&, SchwarzArgs<float>&, const float*) {}

  // z = B r (mode 0) or z += B r (mode 1)
  void schwarz(Level& L, const double* r, double* z, int mode) {
    if (msel || (learned && &L == &lv.back())) {   // uniform levels only (checked at set-up)
      SchwarzArgs<double> a = sz_args<double>(L, L.bk[0], r, z, mode);
      if (msel) {
        // block-diagonal local solves on the selected subdomains only (their supports are disjoint)
        a.sel = msel;
        a.unweighted = 1;
        fill(L.ndof, z, 0.0, st);
        fill(L.nin, L.O, 0.0, st);
      } else {
        add_learned(L, a, r);
      }
      schwarz_solve<double>(L.p, L.m, a, st);
      schwarz_overlap_add<double>(L.p, L.m, a, st);
      return;
    }
    schwarz_t2<double>(L, r, z, mode);
  }
  void schwarz32(Level& L, const float* r, float* z, int mode) { schwarz_t2<float>(L, r, z, mode); }

  // Buckets do not exchange overlap (another degree is zero filled), so the subdomain
  // solves of all buckets may run before or beside any overlap add; every stage is either
  // one launch per bucket or one launch over all buckets.
  template <typename T>
  void schwarz_stage(Level& L, int stage, const T* r, T* z, int mode) {
    if (use_batch(L, stage)) {
      SchwarzArgs<T> a = sz_args<T>(L, L.bk[0], r, z, mode);
      BatchLaunch bl;
      bl.nb = (int)L.bk.size(); bl.ntiles = L.tiles[stage]; bl.grid = batch_grid(L, stage, bl.ntiles); bl.persistent = bl.grid < bl.ntiles;
      if (stage == kStageSolve) schwarz_solve_batched<T>(L.p, a, bdesc<T>(L), bl, st);
      else schwarz_overlap_add_batched<T>(L.p, a, bdesc<T>(L), bl, st);
      return;
    }
    for (const Bucket& b : L.bk) {
      SchwarzArgs<T> a = sz_args<T>(L, b, r, z, mode);
      if (stage == kStageSolve) {
        if constexpr (sizeof(T) == 4) {
          if (matrix_cores() && schwarz_solve_mfma(b.p, b.t->m, a, opt.precision == DGFAS_BF16, st)) continue;
        }
        schwarz_solve<T>(b.p, b.t->m, a, st);
      } else {
        schwarz_overlap_add<T>(b.p, b.t->m, a, st);
      }
    }
  }
  template <typename T>
  void schwarz_t2(Level& L, const T* r, T* z, int mode) {
    if (L.topo) {
      topo_apply<T>(L, r, z, mode);
      return;
    }
    schwarz_stage<T>(L, kStageSolve, r, z, mode);
    schwarz_stage<T>(L, kStageAdd, r, z, mode);
  }
  // unstructured levels: table-driven subdomain solves, then the per-node sums
  template <typename T>
  void topo_apply(Level& L, const T* r, T* z, int mode) {
    const DegTab& t = *L.bk[0].t;
    TopoArgs<T> a;
    a.nel = L.E; a.nrhs = nrhs; a.nt = L.tnt; a.ndof = L.ndof;
    a.r = r; a.z = z; a.mode = mode;
    a.gather = L.tg; a.mptr = L.tmptr; a.midx = L.tmidx; a.var = L.var;
    a.sptr = L.tsptr; a.sslot = L.tsslot;
    if constexpr (sizeof(T) == 8) {
      a.S = t.S; a.ST = t.ST; a.lam = t.lam; a.gco = L.gco; a.Zt = L.Zt; a.scoef = L.tscoef;
    } else {
      a.S = t.S32; a.ST = t.ST32; a.lam = t.lam32; a.gco = L.gco32; a.Zt = L.Zt32; a.scoef = L.tscoef32;
    }
    topo_schwarz_solve<T>(L.ns, a, st);
    topo_schwarz_scatter<T>(a, st);
  }

  // kind 0: out = P in (projection), 1: out (+)= R in (restriction), 2: out += I (in - in2)
  // (prolongation), per element from the fine level's buckets
  void transfer(Level& F, Level& C, int kind, const double* in, const double* in2, double* out, int acc) {
    if (F.hdown) {
      HXferArgs<double> a;
      a.kind = kind; a.ncoarse = C.E; a.children = F.hchild; a.nrhs = nrhs;
      a.stride_f = F.ndof; a.stride_c = C.ndof; a.M = F.hM;
      a.in = in; a.in2 = in2; a.out = out; a.accumulate = acc;
      if (!htransfer<double>(F.p, a, st)) throw Error(DGFAS_EUNSUPPORTED, "no h-transfer kernel for this degree");
      return;
    }
    for (const Bucket& b : F.bk) {
      XferArgs<double> a;
      a.Tm = kind == 0 ? b.Pm : (kind == 1 ? b.Rm : b.Im);
      a.in = in; a.in2 = in2; a.out = out; a.accumulate = acc;
      int n_in, n_out;
      if (F.uniform && C.uniform) {
        a.nel = C.E * nrhs;   // right-hand sides follow each other element-major
        n_in = kind < 2 ? F.n : C.n;
        n_out = kind < 2 ? C.n : F.n;
      } else {
        a.nel = b.nel; a.elist = b.elist; a.nrhs = nrhs;
        if (kind < 2) {
          a.off_in = F.off; a.off_out = C.off; a.stride_in = F.ndof; a.stride_out = C.ndof;
          n_in = b.n; n_out = b.pc + 1;
        } else {
          a.off_in = C.off; a.off_out = F.off; a.stride_in = C.ndof; a.stride_out = F.ndof;
          n_in = b.pc + 1; n_out = b.n;
        }
      }
      if (!tensor3<double>(n_in, n_out, a, st)) throw Error(DGFAS_EUNSUPPORTED, "no transfer kernel for this degree pair");
    }
  }

  // ---------------------------------------------------------------- smoothers
  // r = g - A u into L.r at the start of a smoothing call
  void first_residual(Level& L, const double* u, const double* g) {
    if (rhint && &L == &lv.back() && u == L.u && g == L.g) {
      rhint = false;
      return;
    }
    residual(L, u, g, L.r);
  }

  void was(Level& L, double* u, const double* g, int n) {
    for (int i = 0; i < n; ++i) {
      if (i == 0) first_residual(L, u, g);
      else residual(L, u, g, L.r);
      schwarz(L, L.r, u, 1);
    }
  }

  // Correction-form smoothing in FP32: r = g - A u (FP64); n WAS steps on
  // A du = r in FP32 from du = 0; u += du (FP64).
  void ensure_mixed_vectors(Level& L) {
    const size_t nv = (size_t)L.ndof * nrhs;
    if (!L.r32) L.r32 = own(dalloc<float>(nv));
    if (!L.du32) L.du32 = own(dalloc<float>(nv));
    if (!L.rc32) L.rc32 = own(dalloc<float>(nv));
    if (!L.O32) {
      const size_t nin = (size_t)L.nin * nrhs;
      L.O32 = own(dalloc<float>(nin));
      if (nin) HIPC(hipMemsetAsync(L.O32, 0, nin * sizeof(float), st));
    }
  }

  void was_mixed(Level& L, double* u, const double* g, int n) {
    if (n <= 0) return;
    ensure_mixed_vectors(L);
    first_residual(L, u, g);
    convert<double, float>(L.ndof * nrhs, L.r, L.r32, 0, st);
    schwarz32(L, L.r32, L.du32, 0);
    for (int i = 1; i < n; ++i) {
      residual32(L, L.du32, L.r32, L.rc32);
      schwarz32(L, L.rc32, L.du32, 1);
    }
    convert<float, double>(L.ndof * nrhs, L.du32, u, 1, st);
  }

  // per right-hand side dot products a^T b, synchronously
  std::vector<double> dots_sync(Level& L, const double* a, const double* b) {
    const int nb = reduction_blocks(L.ndof);
    dot_partials<double>(L.ndof, nrhs, a, b, nullptr, partial, nb, st);
    finish(nb, nrhs, partial, nullptr, kOpStore, scal, dotout, st);
    std::vector<double> h(nrhs);
    HIPC(hipMemcpyAsync(h.data(), dotout, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    return h;
  }

  void apply_t(Level& L, const double* u, double* Au) {
    apply(L, u, Au);
    if (mmask) mask_mul(L.ndof, Au, mmask, st);
  }
  void apply_t(Level& L, const float* u, float* Au) { op<float>(L, 1, u, nullptr, Au); }
  void residual_t(Level& L, const double* u, const double* g, double* r) { residual(L, u, g, r); }
  void residual_t(Level& L, const float* u, const float* g, float* r) { residual32(L, u, g, r); }
  void schwarz_t(Level& L, const double* r, double* z, int mode) { schwarz(L, r, z, mode); }
  void schwarz_t(Level& L, const float* r, float* z, int mode) { schwarz32(L, r, z, mode); }

  // Alg. 6 with p = z in the first iteration, every right-hand side with its own scalars.
  // r_max empty: exactly n iterations, no synchronisation; otherwise stop once
  // ||r_k|| <= r_max[k] for every right-hand side k (one synchronisation per iteration).
  // zero_start: x = 0 and r = f without an operator application (correction form).
  // SCG work vectors are allocated at set-up only where the configured cycle runs SCG;
  // other callers (data generation, dgfas_root_solve on any level) get them on first use
  void ensure_scg_vectors(Level& L, bool fp32) {
    const size_t nv = (size_t)L.ndof * nrhs;
    if (!fp32) {
      if (!L.z) L.z = own(dalloc<double>(nv));
      if (!L.pv) L.pv = own(dalloc<double>(nv));
      if (!L.q) L.q = own(dalloc<double>(nv));
      if (!L.r0) L.r0 = own(dalloc<double>(nv));
    } else {
      if (!L.rc32) L.rc32 = own(dalloc<float>(nv));
      if (!L.z32) L.z32 = own(dalloc<float>(nv));
      if (!L.p32) L.p32 = own(dalloc<float>(nv));
      if (!L.q32) L.q32 = own(dalloc<float>(nv));
      if (!L.r0_32) L.r0_32 = own(dalloc<float>(nv));
    }
  }

  static constexpr int kCheck = 4;   // iterations between host convergence checks

  template <typename T>
  int scg(Level& L, T* x, const T* f, int n, const std::vector<double>& r_max, bool* breakdown,
          bool zero_start = false, double* xacc = nullptr) {
    ensure_scg_vectors(L, sizeof(T) == 4);
    const int nb = reduction_blocks(L.ndof);
    const int64_t nv = L.ndof * nrhs;
    T *r, *z, *pv, *q, *r0;
    L.scg_vectors<T>(r, z, pv, q, r0);
    if (zero_start) {
      fill(nv, x, (T)0, st);
      if (f != r) convert<T, T>(nv, f, r, 0, st);   // the caller may have put f in r already
    } else if constexpr (sizeof(T) == 8) {
      if (r == L.r && r_max.empty()) first_residual(L, x, f);
      else residual_t(L, x, f, r);
    } else {
      residual_t(L, x, f, r);
    }
    std::vector<double> h((size_t)8 * nrhs, 0.0);
    if (r_max.empty()) {
      fill((int64_t)8 * nrhs, scal, 0.0, st);
    } else {
      for (int k = 0; k < nrhs; ++k) h[k * 8 + 6] = r_max[k];
      HIPC(hipMemcpyAsync(scal, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
    }
    // semidefinite operator: the root SCG works in the range of A (remark on IPCG, Sec. 4.3.2),
    // projecting its residual and every preconditioned residual (so no fused z^T r there)
    const bool proj = sizeof(T) == 8 && opt.null_space && &L == &lv[0];
    if constexpr (sizeof(T) == 8)
      if (proj) project_mean(L.ndof, nrhs, r, npart, st);
    int it = 0, ran = 0;
    const bool fused = L.zpart && !msel && !proj;
    const bool with_net = learned && &L == &lv.back() && sizeof(T) == 8;
    for (int i = 1; i <= n; ++i) {
      if (fused) {
        // z = B r with z^T r (and z^T (r - r0)) summed by the overlap-add kernel
        SchwarzArgs<T> a = sz_args<T>(L, L.bk[0], r, z, 0);
        if (with_net) add_learned(L, a, r);
        bool done = false;
        if constexpr (sizeof(T) == 4)
          done = matrix_cores() && schwarz_solve_mfma(L.p, L.m, a, opt.precision == DGFAS_BF16, st);
        if (!done) schwarz_solve<T>(L.p, L.m, a, st);
        a.dr = r;
        a.dr0 = i > 1 ? r0 : nullptr;
        a.dotz = L.zpart;
        a.dotz2 = i > 1 ? L.zpart + (size_t)L.nla * nrhs : nullptr;
        schwarz_overlap_add<T>(L.p, L.m, a, st);
        finish(L.nla, nrhs, a.dotz, a.dotz2, i > 1 ? kOpBeta : kOpGamma, scal, nullptr, st, L.nla);
        pupdate<T>(L.ndof, nrhs, z, pv, i > 1 ? x : nullptr, scal, i > 1 ? 0 : 1, st);
      } else if (i > 1) {
        schwarz_t(L, r, z, 0);
        if constexpr (sizeof(T) == 8)
          if (proj) project_mean(L.ndof, nrhs, z, npart, st);
        dot_partials<T>(L.ndof, nrhs, z, r, nullptr, partial, nb, st);
        dot_partials<T>(L.ndof, nrhs, z, r, r0, partial2(), nb, st);
        finish(nb, nrhs, partial, partial2(), kOpBeta, scal, nullptr, st);
        pupdate<T>(L.ndof, nrhs, z, pv, x, scal, 0, st);
      } else {
        schwarz_t(L, r, z, 0);
        if constexpr (sizeof(T) == 8)
          if (proj) project_mean(L.ndof, nrhs, z, npart, st);
        dot_partials<T>(L.ndof, nrhs, z, r, nullptr, partial, nb, st);
        finish(nb, nrhs, partial, nullptr, kOpGamma, scal, nullptr, st);
        pupdate<T>(L.ndof, nrhs, z, pv, nullptr, scal, 1, st);
      }
      if (L.kpart && !mmask) {
        // q = A p with p^T q summed by the operator kernel itself
        OpArgs<T> a = op_args<T>(L, L.bk[0], 1, pv, nullptr, q);
        a.dotp = L.kpart;
        sipg_apply<T>(L.p, a, st);
        finish(L.nlb, nrhs, L.kpart, nullptr, kOpAlpha, scal, nullptr, st, L.nlb);
      } else {
        apply_t(L, pv, q);
        dot_partials<T>(L.ndof, nrhs, pv, q, nullptr, partial, nb, st);
        finish(nb, nrhs, partial, nullptr, kOpAlpha, scal, nullptr, st);
      }
      // r_new = r - alpha q goes to the other residual buffer, which then holds r0; the
      // update u += alpha p rides on the next iteration's p update (or follows the loop)
      // ||r||^2 feeds only the convergence test, so a fixed-count smoothing call skips it
      const bool track = !r_max.empty();
      cg_update<T>(L.ndof, nrhs, r, r0, q, scal, track ? partial : nullptr, nb, st);
      std::swap(r, r0);
      if (track) finish(nb, nrhs, partial, nullptr, kOpNorm2, scal, nullptr, st);
      it = i;
      ran = i;
      // A converged right-hand side is frozen on the device at the iteration where it
      // converged, so the host needs to look only every kCheck iterations: the iterates are
      // those of a check after every iteration, at a fraction of the synchronisations.
      if (!r_max.empty() && (i % kCheck == 0 || i == n)) {
        HIPC(hipMemcpyAsync(h.data(), scal, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        bool done = true, bad = false;
        it = 0;
        for (int k = 0; k < nrhs; ++k) {
          bad = bad || h[k * 8 + 4] != 0.0;
          done = done && (h[k * 8 + 7] != 0.0 || std::sqrt(h[k * 8 + 3]) <= r_max[k]);
          it = std::max(it, (int)h[k * 8 + 5]);
        }
        if (bad) { if (breakdown) *breakdown = true; break; }
        if (done) break;
        it = i;
      }
    }
    if constexpr (sizeof(T) == 4) {
      if (ran && xacc) xupdate_acc(L.ndof, nrhs, x, pv, scal, xacc, st);   // xacc += x + alpha p
      else if (ran) xupdate<T>(L.ndof, nrhs, x, pv, scal, st);
    } else {
      if (ran) xupdate<T>(L.ndof, nrhs, x, pv, scal, st);
    }
    if constexpr (sizeof(T) == 8) {
      if (ran && r_max.empty() && !msel && !mmask) L.rsm = r;
    }
    return it;
  }

  // Correction-form SCG smoothing in FP32: r = g - A u (FP64), n SCG iterations
  // on A du = r in FP32 from du = 0, u += du (FP64).
  void scg_mixed(Level& L, double* u, const double* g, int n) {
    ensure_mixed_vectors(L);
    ensure_scg_vectors(L, true);
    first_residual(L, u, g);
    // the FP32 residual goes straight into the SCG residual buffer, and the last update of the
    // correction straight into u
    convert<double, float>(L.ndof * nrhs, L.r, L.rc32, 0, st);
    scg<float>(L, L.du32, L.rc32, n, {}, nullptr, true, u);
  }

  void smooth(Level& L, double* u, const double* g, int n) {
    L.rsm = nullptr;
    if (n <= 0) return;
    const bool mixed = opt.precision != DGFAS_FP64;
    if (opt.smoother == DGFAS_SCG) {
      if (mixed) scg_mixed(L, u, g, n);
      else scg<double>(L, u, g, n, {}, nullptr);
    } else if (mixed) {
      was_mixed(L, u, g, n);
    } else {
      was(L, u, g, n);
    }
  }

  // root_rtol = 0: exactly root_max_iter SCG iterations with no convergence test, so the root
  // solve needs no host synchronisation and the whole cycle can be captured as one graph
  bool fixed_root() const { return opt.root_rtol == 0.0; }
  // FD contractions of the FP32 smoother on matrix cores (BF16 or FP32 operands)
  bool matrix_cores() const { return opt.precision == DGFAS_BF16 || opt.precision == DGFAS_FP32_MFMA; }

  int root_solve(double* u, const double* g, bool* breakdown) {
    Level& L = lv[0];
    if (fixed_root()) return scg<double>(L, u, g, opt.root_max_iter, {}, breakdown);
    residual(L, u, g, L.r);
    if (opt.null_space) project_mean(L.ndof, nrhs, L.r, npart, st);
    std::vector<double> rmax = dots_sync(L, L.r, L.r);
    bool any = false;
    for (double& v : rmax) {
      v = opt.root_rtol * std::sqrt(v);
      any = any || v > 0.0;
    }
    if (!any) return 0;
    return scg<double>(L, u, g, opt.root_max_iter, rmax, breakdown);
  }

  // Alg. 2 with p-coarsening (per element on mixed-degree levels): the leg above the root
  // solve going down (pre-smoothing, tau-correction), the root solve, the leg going up.
  void vcycle(double* u_top, const double* f_top) {
    const int Lc = (int)lv.size();
    Level& T = lv[Lc - 1];
    double* u_save = T.u;
    const double* g_save = T.g;
    T.u = u_top;
    T.g = const_cast<double*>(f_top);
    bool bd = false;
    leg_down(Lc - 1);
    rhint = false;
    root_solve(lv[0].u, lv[0].g, &bd);
    leg_up(Lc - 1);
    T.u = u_save;
    T.g = const_cast<double*>(g_save);
  }

  // The same cycle with both legs replayed from captured graphs (bitwise the same work); with
  // a fixed-iteration root solve the whole cycle is one graph.
  void vcycle_graphed(double* u_top, const double* f_top) {
    if (!gdown || gu != u_top || gf != f_top || graph_built_epoch != graph_epoch || graph_hint != rhint ||
        graph_ns1 != ns1_top)
      build_graphs(u_top, f_top);
    rhint = false;
    HIPC(hipGraphLaunch(gdown, st));
    if (!fixed_root()) {
      bool bd = false;
      root_solve(lv[0].u, lv[0].g, &bd);
      HIPC(hipGraphLaunch(gup, st));
    }
  }

  // every work vector a leg may touch, allocated before capture
  void prepare_legs() {
    const bool fp32 = opt.precision != DGFAS_FP64;
    if (fixed_root()) ensure_scg_vectors(lv[0], false);
    for (size_t l = 1; l < lv.size(); ++l) {
      Level& L = lv[l];
      if (fp32) ensure_mixed_vectors(L);
      if (opt.smoother == DGFAS_SCG) ensure_scg_vectors(L, fp32);
      if (!fp32 && !L.z) L.z = own(dalloc<double>((size_t)L.ndof * nrhs));
    }
  }

  void build_graphs(double* u_top, const double* f_top) {
    drop_graphs();
    prepare_legs();
    if (!cap) HIPC(hipStreamCreate(&cap));
    HIPC(hipStreamSynchronize(st));
    const int Lc = (int)lv.size();
    Level& T = lv[Lc - 1];
    double* u_save = T.u;
    const double* g_save = T.g;
    hipStream_t saved = st;
    T.u = u_top;
    T.g = const_cast<double*>(f_top);
    const bool hint = rhint;   // the captured down leg starts from r, as the replays will
    st = cap;
    hipGraphExec_t* dst[2] = {&gdown, &gup};
    const bool whole = fixed_root();
    try {
      for (int leg = 0; leg < (whole ? 1 : 2); ++leg) {
        HIPC(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
          if (whole) {
            leg_down(Lc - 1);
            rhint = false;
            bool bd = false;
            root_solve(lv[0].u, lv[0].g, &bd);
            leg_up(Lc - 1);
          } else if (leg == 0) {
            leg_down(Lc - 1);
          } else {
            leg_up(Lc - 1);
          }
        } catch (...) {
          hipGraph_t g = nullptr;
          hipStreamEndCapture(cap, &g);
          if (g) hipGraphDestroy(g);
          throw;
        }
        hipGraph_t g = nullptr;
        HIPC(hipStreamEndCapture(cap, &g));
        const hipError_t e = hipGraphInstantiate(dst[leg], g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        HIPC(e);
      }
    } catch (...) {
      st = saved;
      T.u = u_save;
      T.g = const_cast<double*>(g_save);
      drop_graphs();
      throw;
    }
    st = saved;
    T.u = u_save;
    T.g = const_cast<double*>(g_save);
    gu = u_top;
    gf = f_top;
    graph_built_epoch = graph_epoch;
    graph_hint = hint;
    graph_ns1 = ns1_top;
  }

  // V-cycle on levels 1..top + 1 with lv[top] as the top level (its own u and g); top = 0 is
  // the root solve alone
  void vcycle_sub(int top) {
    bool bd = false;
    if (top > 0) leg_down(top);
    rhint = false;
    root_solve(lv[0].u, lv[0].g, &bd);
    if (top > 0) leg_up(top);
  }

  // Start-up (Sec. 3.3): the coarser levels' right-hand sides f_{l-1} = R f_l go to their g and
  // the start values u_{l-1} = P u_l to their u; then Alg. 4 (FMG: a V-cycle on levels 1..l, then
  // u_{l+1} = I u_l) or Alg. 3 (CMG: root solve, then u_l = I u_{l-1} smoothed with ns0 steps up
  // to level L - 1); the top level receives I u_{L-1}
  void startup(double* u_top, const double* f_top) {
    const int Lc = (int)lv.size();
    if (opt.start == DGFAS_START_NONE) return;
    rhint = false;
    if (Lc == 1) {
      bool bd = false;
      root_solve(u_top, f_top, &bd);
      return;
    }
    for (int l = Lc - 1; l >= 1; --l) {
      Level& F = lv[l];
      Level& C = lv[l - 1];
      transfer(F, C, 1, l == Lc - 1 ? f_top : F.g, nullptr, C.g, 0);
      transfer(F, C, 0, l == Lc - 1 ? u_top : F.u, nullptr, C.u, 0);
    }
    if (opt.start == DGFAS_START_FMG) {
      for (int l = 0; l <= Lc - 2; ++l) {
        vcycle_sub(l);
        transfer(lv[l + 1], lv[l], 2, lv[l].u, nullptr, l + 1 == Lc - 1 ? u_top : lv[l + 1].u, 0);
      }
    } else {
      const int ns0 = opt.ns0 > 0 ? opt.ns0 : opt.ns1 + opt.ns2;
      bool bd = false;
      root_solve(lv[0].u, lv[0].g, &bd);
      for (int l = 1; l <= Lc - 2; ++l) {
        transfer(lv[l], lv[l - 1], 2, lv[l - 1].u, nullptr, lv[l].u, 0);
        smooth(lv[l], lv[l].u, lv[l].g, ns0);
      }
      transfer(lv[Lc - 1], lv[Lc - 2], 2, lv[Lc - 2].u, nullptr, u_top, 0);
    }
  }

  // down leg of a V-cycle whose top level is lv[top]; the finest level takes ns1_top
  // pre-smoothing steps when set (crossover smoothing)
  void leg_down(int top) {
    const int Lc = (int)lv.size();
    for (int l = top; l >= 1; --l) {
      Level& F = lv[l];
      Level& C = lv[l - 1];
      smooth(F, F.u, F.g, (l == Lc - 1 && ns1_top >= 0) ? ns1_top : opt.ns1);
      rhint = false;
      // r = g - A u: an FP64 SCG smoother leaves it as its recurrence residual (the same
      // vector up to rounding), any other smoother has it computed here
      const double* rF = F.rsm;
      if (!rF) {
        residual(F, F.u, F.g, F.r);
        rF = F.r;
      }
      F.rsm = nullptr;
      if (F.lr_down) {
        // local refinement (Alg. 2, eq. helmholtz:fas:rhs): only the twigs take the projected
        // solution and the FAS right-hand side A u + R r; leaves keep theirs
        lr_transfer(F, C, 0, false, F.u, nullptr, C.ubar, 0);                     // ubar^t = P u^a
        copy_rows(C.twig_list, C.ntwig, C.N3, C.ubar, C.u, st);
        apply(C, C.u, C.r);                                                      // A u (active rows)
        lr_transfer(F, C, 1, false, rF, nullptr, C.r, 1);                        //   + R r at twigs
        copy_rows(C.twig_list, C.ntwig, C.N3, C.r, C.g, st);
        continue;
      }
      transfer(F, C, 0, F.u, nullptr, C.ubar, 0);                              // ubar = P u
      HIPC(hipMemcpyAsync(C.u, C.ubar, C.ndof * nrhs * sizeof(double), hipMemcpyDeviceToDevice, st));
      apply(C, C.ubar, C.g);                                                     // g = A ubar
      transfer(F, C, 1, rF, nullptr, C.g, 1);                                    //   + R r
    }
  }

  // transfers of a locally refined level F and the level C below it: kind 0 projection and
  // 1 restriction from the active children into the twig parents, kind 2 prolongation from the
  // twig parents (irregular = false) or the irregular leaf parents (true) to their children
  void lr_transfer(Level& F, Level& C, int kind, bool irregular, const double* in, const double* in2, double* out,
                   int acc) {
    HXferArgs<double> a;
    a.kind = kind;
    a.ncoarse = irregular ? F.nir : F.ntw;
    a.parents = irregular ? F.ir_par : F.tw_par;
    a.children = irregular ? F.ir_ch : F.tw_ch;
    a.nrhs = 1; a.stride_f = F.ndof; a.stride_c = C.ndof; a.M = F.hM;
    a.in = in; a.in2 = in2; a.out = out; a.accumulate = acc;
    if (!htransfer<double>(F.p, a, st)) throw Error(DGFAS_EUNSUPPORTED, "no h-transfer kernel for this degree");
  }

  // FMG start-up on locally refined levels (Alg. 4): stage `top` is a V-cycle on levels
  // 1..top + 1 whose top level takes its own discrete right-hand side on every active element
  // (its twigs act as leaves), then u_{top+2} = I u_{top+1}: active children from their twig
  // parents, frozen children from their leaf parents
  void startup_lr(double* u_top) {
    const int Lc = (int)lv.size();
    for (int top = 0; top <= Lc - 2; ++top) {
      Level& T = lv[top];
      if (T.lr) copy_rows(T.act_list, T.nact, T.N3, T.bfull, T.g, st);
      else HIPC(hipMemcpyAsync(T.g, T.bfull, T.ndof * sizeof(double), hipMemcpyDeviceToDevice, st));
      vcycle_sub(top);
      Level& F = lv[top + 1];
      double* uf = top + 1 == Lc - 1 ? u_top : F.u;
      if (F.lr_down) {
        lr_transfer(F, T, 2, false, T.u, nullptr, uf, 0);
        lr_transfer(F, T, 2, true, T.u, nullptr, uf, 0);
      } else {
        transfer(F, T, 2, T.u, nullptr, uf, 0);
      }
    }
  }

  // composite residual (eq. helmholtz:fas:converged:leaves): sum over the levels of the squared
  // leaf rows of g - A u, with the top level's u and g given
  double composite_norm2(const double* u_top, const double* g_top) {
    double s2 = 0.0;
    const int Lc = (int)lv.size();
    for (int l = 0; l < Lc; ++l) {
      Level& L = lv[l];
      if (!L.nleaf) continue;
      const bool top = l == Lc - 1;
      residual(L, top ? u_top : L.u, top ? g_top : L.g, L.r);
      rows_sumsq(L.leaf_list, L.nleaf, L.N3, L.r, L.sq, st);
      std::vector<double> h = download(L.sq, L.nleaf, st);
      for (double v : h) s2 += v;
    }
    return s2;
  }

  void leg_up(int top) {
    for (int l = 1; l <= top; ++l) {
      Level& F = lv[l];
      Level& C = lv[l - 1];
      if (F.lr_down) {
        lr_transfer(F, C, 2, true, C.u, nullptr, F.u, 0);                      // u^f = I u^l_{l-1}
        lr_transfer(F, C, 2, false, C.u, C.ubar, F.u, 1);                      // u^a += I (u^t - ubar^t)
      } else {
        transfer(F, C, 2, C.u, C.ubar, F.u, 1);                                // u += I (u_c - ubar)
      }
      smooth(F, F.u, F.g, opt.ns2);
    }
  }

  void autotune(const char* path, int reps, double* report);
};

template <typename T>
OpArgs<T> Solver::op_args(Level& L, const Bucket& b, int mode, const T* u, const T* g, T* out) {
  OpArgs<T> a;
  a.E = L.E;
  a.nel = b.nel;
  a.elist = b.elist;
  a.off = L.off;
  a.offF = L.offF;
  a.deg = L.deg;
  if (L.lr) { a.nel = L.nact; a.elist = L.act_list; }
  a.ndof = L.ndof;
  a.nrhs = nrhs;
  a.u = u;
  a.g = g;
  a.out = out;
  a.mode = mode;
  a.nbr = L.nbr;
  a.bc = L.bc;
  a.nfo = L.nfo;
  if (L.nm) {
    a.fmapE = L.mfmapE;
    a.fres = reinterpret_cast<const T*>(L.mfres);
    a.fres_stride = (int64_t)2 * L.nmf * kMortarFaceRes;
  }
  a.kappa = (T)opt.kappa;
  a.inv_wend = (T)b.t->inv_wend;
  if constexpr (sizeof(T) == 8) {
    a.G = L.G; a.WJ = opt.kappa != 0.0 ? L.WJ : nullptr; a.pen = L.pen; a.D = b.t->D;
  } else {
    a.G = L.G32; a.WJ = opt.kappa != 0.0 ? L.WJ32 : nullptr; a.pen = L.pen32; a.D = b.t->D32;
  }
  return a;
}

template <typename T>
SchwarzArgs<T> Solver::sz_args(Level& L, const Bucket& b, const T* r, T* z, int mode) {
  SchwarzArgs<T> a;
  a.E = L.E;
  a.nel = b.nel;
  a.elist = b.elist;
  a.off = L.off;
  a.offO = L.offO;
  a.deg = L.lr ? L.sdeg : L.deg;
  if (L.lr) { a.nel = L.nact; a.elist = L.act_list; }
  a.ndof = L.ndof;
  a.nin = L.nin;
  a.nrhs = nrhs;
  a.r = r;
  a.z = z;
  a.mode = mode;
  a.nb27 = L.nb27;
  a.var = L.var;
  const DegTab& t = *b.t;
  a.map1d = t.map1d;
  if constexpr (sizeof(T) == 8) {
    a.O = inbox64 ? inbox64 : L.O; a.gco = L.gco; a.S = t.S; a.ST = t.ST; a.lam = t.lam; a.W = t.W; a.cinv = L.cinv;
  } else {
    a.O = L.O32; a.gco = L.gco32; a.S = t.S32; a.ST = t.ST32; a.lam = t.lam32; a.W = t.W32; a.cinv = L.cinv32;
  }
  return a;
}

const int kFace[3][2] = {{0, 1}, {2, 3}, {4, 5}};

// Overlap layers at degree p: the option itself, or from delta (Sec. 4.3.1 item 3): the number
// of the neighbour's GLL nodes with (1 + xi)/2 <= delta, its face node included
int overlap_of(const dgfas_options& o, int p) {
  if (o.overlap >= 0) return std::min(o.overlap, p);
  const Gll& g = gll_table(p);
  int m = 0;
  for (int i = 0; i <= p; ++i)
    if (0.5 * (1.0 + g.x[i]) <= o.delta + 1e-14) ++m;
  return std::min(m, p);
}
// (degree, overlap) pairs with Schwarz kernels
bool overlap_supported(int p, int m) {
  return m == 0 || m == 1 || (m == 2 && (p == 4 || p == 8)) || (m == 3 && p == 8);
}

// tables of degree p (built once per solver)
DegTab& deg_tab(Solver& s, int p) {
  auto it = s.tabs.find(p);
  if (it != s.tabs.end()) return it->second;
  hipStream_t st = s.st;
  DegTab& t = s.tabs[p];
  const Gll& gl = gll_table(p);
  t.p = p; t.n = p + 1;
  t.m = overlap_of(s.opt, p);
  t.ns = t.n + 2 * t.m;
  t.inv_wend = 1.0 / gl.w[0];
  t.D = s.own(upload(gl.D, st));
  t.D32 = s.own(upload(to_float(gl.D), st));
  t.w1 = s.own(upload(gl.w, st));
  t.x1 = s.own(upload(gl.x, st));
  // variant tables (left, right) in {I, D, N, I0}^2, zero padded to ns
  const int NS = t.ns, NV = kSides * kSides;
  std::vector<double> S(NV * NS * NS, 0.0), lam(NV * NS, 1.0), W(NV * NS, 0.0);
  std::vector<int> map(NV * NS, -1);
  for (int left = 0; left < kSides; ++left)
    for (int right = 0; right < kSides; ++right) {
      const int v = left * kSides + right;
      Variant1D vt = make_variant_1d(p, t.m, left, right, s.opt.mu_star);
      if (s.opt.weighting == DGFAS_WEIGHT_PLAIN) std::fill(vt.W.begin(), vt.W.end(), 1.0);   // W = I
      for (int i = 0; i < vt.ns; ++i) {
        for (int a = 0; a < vt.ns; ++a) S[v * NS * NS + i * NS + a] = vt.S[i * vt.ns + a];
        lam[v * NS + i] = vt.lam[i];
        W[v * NS + i] = vt.W[i];
        map[v * NS + i] = (vt.delta[i] + 1) * 64 + vt.loc[i];
      }
    }
  std::vector<double> ST(S.size());
  for (int v = 0; v < NV; ++v)
    for (int i = 0; i < NS; ++i)
      for (int a = 0; a < NS; ++a) ST[v * NS * NS + a * NS + i] = S[v * NS * NS + i * NS + a];
  t.S = s.own(upload(S, st)); t.S32 = s.own(upload(to_float(S), st));
  t.ST = s.own(upload(ST, st)); t.ST32 = s.own(upload(to_float(ST), st));
  t.lam = s.own(upload(lam, st)); t.lam32 = s.own(upload(to_float(lam), st));
  t.W = s.own(upload(W, st)); t.W32 = s.own(upload(to_float(W), st));
  t.map1d = s.own(upload(map, st));
  t.h_W = W;
  t.h_map = map;
  return t;
}

// Level set-up from per-element degrees and device coordinates (element e at 3 off[e]).
void build_level(Solver& s, Level& L, const std::vector<int>& deg, const double* dX, double* dNu) {
  hipStream_t st = s.st;
  const int E = L.E;   // set by the caller with the level's topology
  L.h_deg = deg;
  L.p = *std::max_element(deg.begin(), deg.end());
  L.uniform = *std::min_element(deg.begin(), deg.end()) == L.p;
  L.n = L.p + 1; L.N2 = L.n * L.n; L.N3 = L.N2 * L.n;
  L.m = overlap_of(s.opt, L.p);
  L.ns = L.n + 2 * L.m;
  L.inv_wend = 1.0 / gll_table(L.p).w[0];
  // element-major layout with offsets
  std::vector<int64_t> off(E), offF(E), offO(E);
  int64_t nd = 0, nf = 0, no = 0;
  for (int e = 0; e < E; ++e) {
    const int n = deg[e] + 1;
    off[e] = nd; offF[e] = nf; offO[e] = no;
    nd += (int64_t)n * n * n;
    nf += 6 * (int64_t)n * n;
    no += overlap_size(deg[e], overlap_of(s.opt, deg[e]));
  }
  L.ndof = nd; L.nfs = nf; L.nin = no;
  L.h_off = off;
  if (!L.uniform) {
    L.deg = s.own(upload(deg, st));
    L.off = s.own(upload(off, st));
    L.offF = s.own(upload(offF, st));
    L.offO = s.own(upload(offO, st));
  }
  // degree buckets
  for (int p = 1; p <= 8; ++p) {
    Bucket b;
    for (int e = 0; e < E; ++e)
      if (deg[e] == p) b.h_elist.push_back(e);
    if (b.h_elist.empty()) continue;
    b.p = p; b.n = p + 1; b.nel = (int)b.h_elist.size();
    if (!s.rank.empty() && L.E == s.E)
      std::stable_sort(b.h_elist.begin(), b.h_elist.end(), [&](int x, int y) { return s.rank[x] < s.rank[y]; });
    if (!L.uniform || (!s.rank.empty() && L.E == s.E)) b.elist = s.own(upload(b.h_elist, st));
    b.t = &deg_tab(s, p);
    L.all_m1 = L.all_m1 && b.t->m == 1;
    L.bk.push_back(std::move(b));
  }
  // local refinement: the sweep kernels take the active elements (frozen ones keep their
  // values, their rows are never written); the Schwarz kernels see a frozen element as one of
  // another degree (no overlap into it, zero fill, no scatter)
  if (L.lr) {
    std::vector<int> act, leaf, twig, sd(E);
    for (int e = 0; e < E; ++e) {
      const int8_t c = L.h_cls[e];
      if (c != kFrozen) act.push_back(e);
      if (c == kLeaf) leaf.push_back(e);
      if (c == kTwig) twig.push_back(e);
      sd[e] = c == kFrozen ? -1 : deg[e];
    }
    L.nact = (int)act.size(); L.nleaf = (int)leaf.size(); L.ntwig = (int)twig.size();
    L.act_list = s.own(upload(act, st));
    if (L.nleaf) L.leaf_list = s.own(upload(leaf, st));
    if (L.ntwig) L.twig_list = s.own(upload(twig, st));
    L.sdeg = s.own(upload(sd, st));
    if (L.nleaf) L.sq = s.own(dalloc<double>(L.nleaf));
  }
  // degree histogram and the one-launch work lists (largest degree first)
  for (const Bucket& b : L.bk) L.hist += std::to_string(b.p) + ":" + std::to_string(b.nel) + ",";
  if (!L.uniform) {
    std::vector<BucketDesc<double>> d64;
    std::vector<BucketDesc<float>> d32;
    int t0[3] = {0, 0, 0};
    for (int k = (int)L.bk.size() - 1; k >= 0; --k) {
      const Bucket& b = L.bk[k];
      const DegTab& t = *b.t;
      BucketDesc<double> x;
      BucketDesc<float> y;
      x.p = y.p = b.p; x.m = y.m = t.m; x.nel = y.nel = b.nel;
      x.elist = y.elist = b.elist;
      for (int sg = 0; sg < 3; ++sg) {
        x.tile0[sg] = y.tile0[sg] = t0[sg];
        t0[sg] += stage_tiles(sg, b.p, b.nel, s.nrhs);
      }
      x.D = t.D; x.S = t.S; x.ST = t.ST; x.lam = t.lam; x.W = t.W; x.map1d = t.map1d; x.inv_wend = t.inv_wend;
      y.D = t.D32; y.S = t.S32; y.ST = t.ST32; y.lam = t.lam32; y.W = t.W32; y.map1d = t.map1d;
      y.inv_wend = (float)t.inv_wend;
      d64.push_back(x);
      d32.push_back(y);
    }
    for (int sg = 0; sg < 3; ++sg) L.tiles[sg] = t0[sg];
    L.bd64 = s.own(upload(d64, st));
    L.bd32 = s.own(upload(d32, st));
  }
  // elements with a face to another degree
  if (!L.uniform) {
    std::vector<int> ml;
    for (int e = 0; e < E; ++e) {
      bool any = false;
      for (int f = 0; f < 6; ++f) {
        const int en = L.h_nbr[e * 6 + f];
        any = any || (en >= 0 && deg[en] != deg[e]);
      }
      if (any) ml.push_back(e);
    }
    L.nm = (int)ml.size();
    if (L.nm) {
      // one task per face, listed from its lower-id side; slot 2k is that side's result,
      // 2k + 1 the other side's
      std::vector<int64_t> fd;
      std::vector<int> fm((size_t)E * 6, -1);
      for (int li = 0; li < L.nm; ++li) {
        const int e = ml[li];
        for (int f = 0; f < 6; ++f) {
          const int en = L.h_nbr[e * 6 + f];
          if (en >= 0 && deg[en] != deg[e] && e < en) {
            const int k = (int)(fd.size() / 8);
            fm[(size_t)e * 6 + f] = 2 * k;
            fm[(size_t)en * 6 + (f ^ 1)] = 2 * k + 1;
            const int64_t d[8] = {(int64_t)e * 6 + f, en, deg[e], deg[en], off[e], offF[e], off[en], offF[en]};
            fd.insert(fd.end(), d, d + 8);
          }
        }
      }
      L.nmf = (int)(fd.size() / 8);
      L.mfdesc = s.own(upload(fd, st));
      L.mfmapE = s.own(upload(fm, st));
      s.reserve(L.mfres, (size_t)s.nrhs * 2 * L.nmf * kMortarFaceRes);
    }
  }
  // geometry per bucket
  L.G = s.own(dalloc<double>(6 * L.ndof));
  L.WJ = s.own(dalloc<double>(L.ndof));
  L.ws = s.own(dalloc<double>(L.nfs));
  L.pen = s.own(dalloc<double>(L.nfs));
  L.muf = s.own(dalloc<double>((size_t)E * 6));
  L.vol = s.own(dalloc<double>(E));
  L.area = s.own(dalloc<double>((size_t)E * 6));
  L.lin = s.own(dalloc<double>((size_t)E * 9));
  L.nun = dNu;
  if (dNu) L.nuavg = s.own(dalloc<double>(E));
  int* bad = s.own(dalloc<int>(1));
  HIPC(hipMemsetAsync(bad, 0, sizeof(int), st));
  for (const Bucket& b : L.bk) {
    GeoArgs g;
    g.nel = b.nel; g.elist = b.elist; g.off = L.off; g.offF = L.offF; g.ndof = L.ndof; g.X = dX;
    g.G = L.G; g.WJ = L.WJ; g.ws = L.ws; g.vol = L.vol; g.area = L.area; g.lin = L.lin; g.bad = bad;
    g.nun = L.nun; g.nuavg = L.nuavg;
    geometry(b.p, g, b.t->D, b.t->w1, b.t->x1, s.opt.nu, st);
    HIPC(hipGetLastError());
  }
  penalty(E, L.p, L.deg, L.offF, s.opt.mu_star, s.opt.nu, L.nun, L.nbr, L.nfo, L.bc, L.vol, L.area, L.ws, L.pen,
          L.muf, st);
  HIPC(hipGetLastError());
  int hbad = 0;
  HIPC(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (hbad) throw Error(DGFAS_EINVAL, "element map with det J <= 0 at degree " + std::to_string(L.p));
  // FP32 copies for the correction-form smoother
  L.G32 = s.own(dalloc<float>(6 * L.ndof));
  L.WJ32 = s.own(dalloc<float>(L.ndof));
  L.pen32 = s.own(dalloc<float>(L.nfs));
  convert<double, float>(6 * L.ndof, L.G, L.G32, 0, st);
  convert<double, float>(L.ndof, L.WJ, L.WJ32, 0, st);
  convert<double, float>(L.nfs, L.pen, L.pen32, 0, st);

  // surrogate cuboid (Sec. 4.3.1 steps 1-3): Delta x_b = 2|a_b| (vol / prod)^(1/3)
  std::vector<double> vol = download(L.vol, E, st), lin = download(L.lin, (size_t)E * 9, st);
  // the surrogate's nu: the element average of a nodal field (Sec. 4.3.1), else the scalar
  std::vector<double> nue = L.nuavg ? download(L.nuavg, E, st) : std::vector<double>(E, s.opt.nu);
  for (int e = 0; e < E; ++e)
    if (!(nue[e] > 0))
      throw Error(DGFAS_EINVAL, "the element average of nu must be positive (degree " + std::to_string(L.p) + ")");
  std::vector<double> gco((size_t)E * 4);
  for (int e = 0; e < E; ++e) {
    double ell[3];
    for (int b = 0; b < 3; ++b) {
      double s2 = 0;
      for (int a = 0; a < 3; ++a) s2 += lin[e * 9 + a * 3 + b] * lin[e * 9 + a * 3 + b];
      ell[b] = 2.0 * std::sqrt(s2);
    }
    const double sc = std::cbrt(vol[e] / (ell[0] * ell[1] * ell[2]));
    const double dx[3] = {ell[0] * sc, ell[1] * sc, ell[2] * sc};
    gco[e * 4 + 0] = s.opt.kappa * dx[0] * dx[1] * dx[2] / 8.0;
    gco[e * 4 + 1] = nue[e] * dx[1] * dx[2] / (2.0 * dx[0]);
    gco[e * 4 + 2] = nue[e] * dx[2] * dx[0] / (2.0 * dx[1]);
    gco[e * 4 + 3] = nue[e] * dx[0] * dx[1] / (2.0 * dx[2]);
  }
  L.gco = s.own(upload(gco, st));
  {
    std::vector<double> j9((size_t)E * 9);
    for (int e = 0; e < E; ++e) {
      const double* A = &lin[e * 9];   // A[a][b] = coefficient of coordinate a along xi_b
      const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                         A[2] * (A[3] * A[7] - A[4] * A[6]);
      const double sc = 1.0 / std::cbrt(det);
      for (int q = 0; q < 9; ++q) j9[e * 9 + q] = A[q] * sc;
    }
    L.J9 = s.own(upload(j9, st));
  }
  L.gco32 = s.own(upload(to_float(gco), st));

  // per element: variant code per direction and the 27-neighbourhood; a side toward an
  // element of another degree takes the no-overlap interior variant
  std::vector<int8_t> var((size_t)E * 3);
  std::vector<int> nb27((size_t)E * 27, -1);
  for (int e = 0; e < E; ++e) {
    for (int d = 0; d < 3; ++d) {
      int code[2];
      for (int sd = 0; sd < 2; ++sd) {
        const int f = kFace[d][sd];
        const int en = L.h_nbr[e * 6 + f];
        const bool frozen_nb = L.lr && en >= 0 && L.h_cls[en] == kFrozen;
        if (en >= 0) code[sd] = deg[en] == deg[e] && !frozen_nb ? kInterior : kInteriorNoOverlap;
        else code[sd] = L.h_bc[e * 6 + f] == DGFAS_NEUMANN ? kNeumann : kDirichlet;
      }
      var[e * 3 + d] = (int8_t)(code[0] * kSides + code[1]);
    }
    for (int d3 = -1; d3 <= 1; ++d3)
      for (int d2 = -1; d2 <= 1; ++d2)
        for (int d1 = -1; d1 <= 1; ++d1) {
          int cur = e;
          const int dd[3] = {d1, d2, d3};
          for (int d = 0; d < 3 && cur >= 0; ++d)
            if (dd[d]) cur = L.h_nbr[cur * 6 + kFace[d][dd[d] > 0]];
          nb27[e * 27 + (d3 + 1) * 9 + (d2 + 1) * 3 + (d1 + 1)] = cur;
        }
  }
  L.var = s.own(upload(var, st));
  L.nb27 = s.own(upload(nb27, st));
  L.h_nb27 = nb27;
  // unstructured level: the subdomain slot tables (every slot's node, zero or merged nodes) and
  // the per-node contribution lists with the normalised weights
  if (L.topo) {
    const DegTab& t = deg_tab(s, L.p);
    TopoMesh tm;
    tm.E = E; tm.n = L.n; tm.nbr = L.h_nbr.data(); tm.nface = L.h_nface.data(); tm.norient = L.h_norient.data();
    TopoTables T;
    try {
      T = topo_tables(tm, t.ns, var.data(), t.h_map.data(), t.h_W.data(), s.opt.weighting == DGFAS_WEIGHT_QUINTIC);
    } catch (const std::runtime_error& x) {
      throw Error(DGFAS_EINVAL, std::string("unstructured mesh: ") + x.what());
    }
    L.tnt = T.nt;
    for (int k = 0; k < 5; ++k) L.tblocks[k] = T.blocks[k];
    L.tg = s.own(upload(T.gather, st));
    L.tmptr = s.own(upload(T.mptr, st));
    if (!T.midx.empty()) L.tmidx = s.own(upload(T.midx, st));
    L.tsptr = s.own(upload(T.sptr, st));
    L.tsslot = s.own(upload(T.sslot, st));
    L.tscoef = s.own(upload(T.scoef, st));
    if (s.opt.precision != DGFAS_FP64) L.tscoef32 = s.own(upload(to_float(T.scoef), st));
  }
  // Weight sum C = sum_s R_s^T W_s R_s 1 at every node.  Near a degree jump the subdomains that
  // reach a node can disagree about who covers it (neighbours of another degree are zero filled),
  // so the corrections are normalised by C there (C > 0: the own subdomain always covers a node)
  // (a frozen neighbour is treated as one of another degree; frozen nodes get no correction)
  auto frozen = [&](int e) { return L.lr && L.h_cls[e] == kFrozen; };
  if ((!L.uniform || L.lr) && L.m > 0 && s.opt.weighting == DGFAS_WEIGHT_QUINTIC) {
    std::vector<double> C((size_t)L.ndof, 0.0);
    for (int e = 0; e < E; ++e) {
      if (frozen(e)) continue;
      const DegTab& t = deg_tab(s, deg[e]);
      const int n = t.n, NS = t.ns;
      const int* mp[3];
      const double* wp[3];
      for (int d = 0; d < 3; ++d) {
        mp[d] = &t.h_map[(size_t)var[e * 3 + d] * NS];
        wp[d] = &t.h_W[(size_t)var[e * 3 + d] * NS];
      }
      for (int s3 = 0; s3 < NS; ++s3)
        for (int s2 = 0; s2 < NS; ++s2)
          for (int s1 = 0; s1 < NS; ++s1) {
            const int m1 = mp[0][s1], m2 = mp[1][s2], m3 = mp[2][s3];
            if (m1 < 0 || m2 < 0 || m3 < 0) continue;
            const int nb = nb27[(size_t)e * 27 + (m3 >> 6) * 9 + (m2 >> 6) * 3 + (m1 >> 6)];
            if (nb < 0 || deg[nb] != deg[e] || frozen(nb)) continue;
            C[off[nb] + ((m3 & 63) * n + (m2 & 63)) * n + (m1 & 63)] += wp[0][s1] * wp[1][s2] * wp[2][s3];
          }
    }
    bool all_one = true;
    for (int e = 0; e < E; ++e) {
      const int64_t n3 = (int64_t)(deg[e] + 1) * (deg[e] + 1) * (deg[e] + 1);
      for (int64_t q = off[e]; q < off[e] + n3; ++q) {
        double& c = C[q];
        if (frozen(e)) { c = 1.0; continue; }
        if (!(c > 0)) throw Error(DGFAS_EINVAL, "node without a covering subdomain");
        all_one = all_one && c == 1.0;
        c = 1.0 / c;
      }
    }
    if (!all_one) {
      L.cinv = s.own(upload(C, st));
      L.cinv32 = s.own(upload(to_float(C), st));
    }
  }
  // Per-call scratch of the configured cycle: reserved in the workspace, which is laid out
  // once every level is built.  Inbox regions of absent neighbours (and of neighbours of
  // another degree) are never written and must read as zero.
  const size_t nin = (size_t)L.nin * s.nrhs;
  const bool fp32 = s.opt.precision != DGFAS_FP64;
  if (L.topo) {
    // the stored subdomain solutions replace the overlap inbox; SCG takes its dot products
    // from separate reductions (no fused partial sums)
    s.reserve(L.Zt, (size_t)E * L.tnt * s.nrhs);
    if (fp32) s.reserve(L.Zt32, (size_t)E * L.tnt * s.nrhs);
  } else {
    s.reserve(L.O, nin, true);
    if (fp32) s.reserve(L.O32, nin, true);
  }
  if (L.uniform) {
    const int nsweep = L.lr ? L.nact : E;   // elements the sweep kernels take
    L.nlb = stage_tiles(kStageOp, L.p, nsweep, 1);
    s.reserve(L.kpart, (size_t)L.nlb * s.nrhs);
    if (L.m > 0 && !L.topo) {
      L.nla = stage_tiles(kStageAdd, L.p, nsweep, 1);
      s.reserve(L.zpart, (size_t)2 * L.nla * s.nrhs);
    }
  }
  // work vectors
  // (on a locally refined level the kernels never write frozen rows, which must read as zero)
  const size_t nv = (size_t)L.ndof * s.nrhs;
  s.reserve(L.r, nv, L.lr);
  const bool scg_here = s.opt.smoother == DGFAS_SCG || &L == &s.lv[0];
  const bool dbl_scg = scg_here && !(fp32 && &L != &s.lv[0]);
  if (dbl_scg || !fp32) s.reserve(L.z, nv, L.lr);
  if (dbl_scg) {
    s.reserve(L.pv, nv, L.lr);
    s.reserve(L.q, nv, L.lr);
    s.reserve(L.r0, nv, L.lr);
  }
  if (fp32 && &L != &s.lv[0]) {
    s.reserve(L.r32, nv);
    s.reserve(L.du32, nv);
    s.reserve(L.rc32, nv);
    if (s.opt.smoother == DGFAS_SCG) {
      s.reserve(L.z32, nv);
      s.reserve(L.p32, nv);
      s.reserve(L.q32, nv);
      s.reserve(L.r0_32, nv);
    }
  }
  HIPC(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------------- autotuner
namespace {

// flat JSON object of string keys and integer values (the autotuner cache)
std::map<std::string, int> read_cache(const char* path) {
  std::map<std::string, int> m;
  if (!path) return m;
  std::ifstream in(path);
  if (!in) return m;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while ((i = t.find('"', i)) != std::string::npos) {
    const size_t j = t.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = t.substr(i + 1, j - i - 1);
    const size_t c = t.find(':', j);
    if (c == std::string::npos) break;
    m[key] = std::atoi(t.c_str() + c + 1);
    i = t.find_first_of(",}", c);
    if (i == std::string::npos) break;
  }
  return m;
}

void write_cache(const char* path, const std::map<std::string, int>& m) {
  if (!path) return;
  std::ofstream out(path);
  if (!out) throw Error(DGFAS_EINVAL, std::string("cannot write the autotuner cache ") + path);
  out << "{\n";
  size_t k = 0;
  for (const auto& kv : m) out << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
  out << "}\n";
}

}  // namespace

void Solver::autotune(const char* path, int reps, double* report) {
  if (reps < 1) throw Error(DGFAS_EINVAL, "reps must be >= 1");
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPC(hipGetDeviceProperties(&prop, dev));
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  std::map<std::string, int> cache = read_cache(path);
  const char* stage_name[3] = {"operator", "solve", "add"};
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  double *x = nullptr, *y = nullptr, *w = nullptr;
  auto cleanup = [&]() {
    force_batch = -1;
    hipStreamSynchronize(st);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (x) hipFree(x);
    if (y) hipFree(y);
    if (w) hipFree(w);
  };
  try {
    for (size_t li = 0; li < lv.size(); ++li) {
      Level& L = lv[li];
      for (int sg = 0; sg < 3; ++sg)
        if (report)
          for (int v = 0; v < 3; ++v) report[(li * 3 + sg) * 3 + v] = 0.0;
      if (L.uniform || L.bk.size() < 2) continue;
      const size_t nv = (size_t)L.ndof * nrhs;
      if (x) { hipStreamSynchronize(st); hipFree(x); hipFree(y); hipFree(w); x = y = w = nullptr; }
      x = dalloc<double>(nv);
      y = dalloc<double>(nv);
      w = dalloc<double>(nv);
      fill((int64_t)nv, x, 0.5, st);
      fill((int64_t)nv, y, 0.25, st);
      for (int sg = 0; sg < 3; ++sg) {
        static const char* const kPrec[4] = {"fp64", "fp32", "bf16", "fp32mfma"};
        const std::string key = arch + "|" + L.hist + "|" + kPrec[opt.precision] + "|rhs" +
                                std::to_string(nrhs) + "|" + stage_name[sg];
        if (sg != kStageOp && !L.all_m1) continue;
        auto it = cache.find(key);
        if (it != cache.end()) {
          L.one_launch[sg] = it->second;
          continue;
        }
        double med[3];
        for (int v = 0; v < 3; ++v) {
          force_batch = v;
          auto run = [&]() {
            if (sg == kStageOp) op<double>(L, 0, x, y, w);
            else schwarz_stage<double>(L, sg, x, w, 1);
          };
          run();   // warm-up
          std::vector<double> ts;
          for (int k = 0; k < reps; ++k) {
            HIPC(hipEventRecord(e0, st));
            run();
            HIPC(hipEventRecord(e1, st));
            HIPC(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            ts.push_back(ms);
          }
          std::sort(ts.begin(), ts.end());
          med[v] = ts[ts.size() / 2];
          HIPC(hipGetLastError());
        }
        force_batch = -1;
        int best = 0;
        for (int v = 1; v < 3; ++v)
          if (med[v] < med[best]) best = v;
        L.one_launch[sg] = best;
        cache[key] = best;
        if (report)
          for (int v = 0; v < 3; ++v) report[(li * 3 + sg) * 3 + v] = med[v];
      }
    }
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
  write_cache(path, cache);
  opt.batch = DGFAS_BATCH_TUNED;
  ++graph_epoch;
}

void validate(const dgfas_mesh_desc* m, const dgfas_options* o) {
  if (!m || !o) throw Error(DGFAS_EINVAL, "null mesh or options");
  if (m->n_elem <= 0 || !m->degree || !m->coords || !m->face_nbr || !m->face_bc)
    throw Error(DGFAS_EINVAL, "mesh arrays missing or n_elem <= 0");
  for (int e = 0; e < m->n_elem; ++e)
    if (m->degree[e] < 1 || m->degree[e] > 8) throw Error(DGFAS_EUNSUPPORTED, "degree must be 1..8");
  for (int e = 0; e < m->n_elem; ++e)
    for (int f = 0; f < 6; ++f) {
      const int en = m->face_nbr[e * 6 + f];
      if (en >= m->n_elem) throw Error(DGFAS_EINVAL, "face neighbour out of range");
      if (en >= 0 && !m->face_nbr_face && m->face_nbr[en * 6 + (f ^ 1)] != e)
        throw Error(DGFAS_EUNSUPPORTED, "face neighbours must be aligned and mutual (or give face_nbr_face)");
      if (en < 0 && m->face_bc[e * 6 + f] != DGFAS_DIRICHLET && m->face_bc[e * 6 + f] != DGFAS_NEUMANN)
        throw Error(DGFAS_EINVAL, "boundary face without a Dirichlet/Neumann code");
    }
  if (!(o->nu > 0) || !(o->kappa >= 0) || !(o->mu_star > 0)) throw Error(DGFAS_EINVAL, "bad coefficients");
  if (m->face_orient && !m->face_nbr_face) throw Error(DGFAS_EINVAL, "face_orient needs face_nbr_face");
  if (m->face_nbr_face) {
    for (int e = 1; e < m->n_elem; ++e)
      if (m->degree[e] != m->degree[0]) throw Error(DGFAS_EUNSUPPORTED, "an unstructured mesh needs one degree");
    if (o->h_levels > 0 || o->local_steps > 0 || o->precision == DGFAS_BF16 || o->precision == DGFAS_FP32_MFMA)
      throw Error(DGFAS_EUNSUPPORTED, "unstructured meshes run without h_levels, local_steps and matrix-core "
                                      "precisions");
    TopoMesh tm;
    tm.E = m->n_elem; tm.n = m->degree[0] + 1; tm.nbr = m->face_nbr; tm.nface = m->face_nbr_face;
    tm.norient = m->face_orient;
    const std::string bad = topo_check(tm);
    if (!bad.empty()) throw Error(DGFAS_EINVAL, bad);
  }
  if (m->nu_nodal) {
    const int p = m->degree[0];
    for (int e = 1; e < m->n_elem; ++e)
      if (m->degree[e] != p) throw Error(DGFAS_EUNSUPPORTED, "a nodal nu needs one degree on the mesh");
    const int64_t n = (int64_t)m->n_elem * (p + 1) * (p + 1) * (p + 1);
    for (int64_t q = 0; q < n; ++q)
      if (!(m->nu_nodal[q] >= 0) || !std::isfinite(m->nu_nodal[q]))
        throw Error(DGFAS_EINVAL, "nodal nu must be finite and >= 0");
  }
  if (o->overlap < 0 && !(o->delta >= 0.0 && o->delta < 1.0)) throw Error(DGFAS_EINVAL, "delta must be in [0, 1)");
  // every degree on every level (p -> max(1, p / 2) per element) needs a kernel for its overlap
  {
    bool seen[9] = {false};
    for (int e = 0; e < m->n_elem; ++e)
      for (int q = m->degree[e];; q = std::max(1, q / 2)) {
        seen[q] = true;
        if (q == 1) break;
      }
    for (int q = 1; q <= 8; ++q)
      if (seen[q] && !overlap_supported(q, overlap_of(*o, q)))
        throw Error(DGFAS_EUNSUPPORTED, "no Schwarz kernel for degree " + std::to_string(q) + " with overlap " +
                                            std::to_string(overlap_of(*o, q)));
  }
  if (o->weighting != DGFAS_WEIGHT_QUINTIC && o->weighting != DGFAS_WEIGHT_PLAIN)
    throw Error(DGFAS_EINVAL, "unknown weighting");
  if (o->projection != DGFAS_PROJECT_INTERP && o->projection != DGFAS_PROJECT_L2)
    throw Error(DGFAS_EINVAL, "unknown projection");
  if (o->start != DGFAS_START_NONE && o->start != DGFAS_START_CMG && o->start != DGFAS_START_FMG)
    throw Error(DGFAS_EINVAL, "unknown start-up");
  if (o->nsc > 0 && o->nsc < o->ns2) throw Error(DGFAS_EINVAL, "nsc must be >= ns2 (or <= 0 for none)");
  if (o->h_levels < 0 || o->h_levels > 8) throw Error(DGFAS_EINVAL, "h_levels must be 0..8");
  if (o->local_steps < 0 || o->local_steps > 8) throw Error(DGFAS_EINVAL, "local_steps must be 0..8");
  if (o->null_space != 0 && o->null_space != 1) throw Error(DGFAS_EINVAL, "null_space must be 0 or 1");
  if (o->null_space && (o->kappa != 0.0 || o->local_steps > 0))
    throw Error(DGFAS_EINVAL, "null_space needs kappa = 0 and no local refinement");
  if (o->local_steps > 0) {
    if (!m->refine_count || !m->refine_list) throw Error(DGFAS_EINVAL, "local refinement needs refine_count and refine_list");
    for (int e = 1; e < m->n_elem; ++e)
      if (m->degree[e] != m->degree[0]) throw Error(DGFAS_EUNSUPPORTED, "local refinement needs one degree");
    if (o->h_levels > 0 || o->n_rhs != 1 || o->precision != DGFAS_FP64 || o->start == DGFAS_START_CMG ||
        o->graph != 0 || m->nu_nodal || o->nsc > 0 || o->order != DGFAS_ORDER_NATURAL)
      throw Error(DGFAS_EUNSUPPORTED, "local refinement runs FP64, one right-hand side, plain V-cycles, natural "
                                      "order, constant nu and no h_levels");
  }
  if (o->h_only != 0 && o->h_only != 1) throw Error(DGFAS_EINVAL, "h_only must be 0 or 1");
  if (o->h_levels > 0) {
    // h-coarsening needs one degree and a box numbering e = ex + nx (ey + ny ez) whose dimensions
    // halve h_levels times; the face neighbours must be those of the box (or its periodic wraps)
    const int nx = m->box[0], ny = m->box[1], nz = m->box[2];
    if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz != m->n_elem)
      throw Error(DGFAS_EINVAL, "h-coarsening needs box dimensions with nx ny nz = n_elem");
    const int div = 1 << o->h_levels;
    if (nx % div || ny % div || nz % div)
      throw Error(DGFAS_EINVAL, "box dimensions must be divisible by 2^h_levels");
    for (int e = 0; e < m->n_elem; ++e) {
      if (m->degree[e] != m->degree[0]) throw Error(DGFAS_EUNSUPPORTED, "h-coarsening needs one degree");
      const int c[3] = {e % nx, (e / nx) % ny, e / (nx * ny)}, dim[3] = {nx, ny, nz};
      for (int f = 0; f < 6; ++f) {
        const int ax = f >> 1, dir = (f & 1) ? 1 : -1;
        int cc[3] = {c[0], c[1], c[2]};
        cc[ax] = (cc[ax] + dir + dim[ax]) % dim[ax];
        const int en = m->face_nbr[e * 6 + f], box_nb = cc[0] + nx * (cc[1] + ny * cc[2]);
        const bool edge = (dir < 0 && c[ax] == 0) || (dir > 0 && c[ax] == dim[ax] - 1);
        if (en >= 0 ? en != box_nb : !edge)
          throw Error(DGFAS_EINVAL, "face neighbours do not follow the box numbering");
      }
    }
    if (o->order == DGFAS_ORDER_MORTON) throw Error(DGFAS_EUNSUPPORTED, "Morton order with h-coarsening");
  }
  if (o->smoother != DGFAS_WAS && o->smoother != DGFAS_SCG) throw Error(DGFAS_EINVAL, "unknown smoother");
  if (o->ns1 < 0 || o->ns2 < 0 || o->root_max_iter < 1) throw Error(DGFAS_EINVAL, "bad step counts");
  if (!(o->root_rtol >= 0) || !std::isfinite(o->root_rtol)) throw Error(DGFAS_EINVAL, "root_rtol must be >= 0");
  if (o->precision != DGFAS_FP64 && o->precision != DGFAS_FP32 && o->precision != DGFAS_BF16 &&
      o->precision != DGFAS_FP32_MFMA)
    throw Error(DGFAS_EINVAL, "unknown precision");
  if (o->n_rhs < 1 || o->n_rhs > 64) throw Error(DGFAS_EINVAL, "n_rhs must be 1..64");
  if (o->batch < DGFAS_BATCH_PER_DEGREE || o->batch > DGFAS_BATCH_PERSISTENT) throw Error(DGFAS_EINVAL, "unknown batch mode");
  if (o->graph != 0 && o->graph != 1) throw Error(DGFAS_EINVAL, "graph must be 0 or 1");
  if (o->order != DGFAS_ORDER_NATURAL && o->order != DGFAS_ORDER_MORTON) throw Error(DGFAS_EINVAL, "unknown order");
  if ((int64_t)m->n_elem * o->n_rhs > (int64_t)1 << 30) throw Error(DGFAS_EUNSUPPORTED, "n_elem * n_rhs too large");
}

// Morton (Z-order) rank of the element centroids on a 2^10 grid over their bounding box
std::vector<int64_t> morton_rank(const dgfas_mesh_desc* m) {
  const int E = m->n_elem;
  std::vector<double> c((size_t)E * 3);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  size_t o = 0;
  for (int e = 0; e < E; ++e) {
    const int n = m->degree[e] + 1, n3 = n * n * n;
    for (int a = 0; a < 3; ++a) {
      double sum = 0;
      for (int q = 0; q < n3; ++q) sum += m->coords[o + (size_t)a * n3 + q];
      c[e * 3 + a] = sum / n3;
      lo[a] = std::min(lo[a], c[e * 3 + a]);
      hi[a] = std::max(hi[a], c[e * 3 + a]);
    }
    o += (size_t)3 * n3;
  }
  std::vector<int64_t> key(E);
  for (int e = 0; e < E; ++e) {
    uint64_t k = 0;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
      const double w = hi[a] > lo[a] ? (c[e * 3 + a] - lo[a]) / (hi[a] - lo[a]) : 0.0;
      q[a] = (uint32_t)std::min(1023.0, std::max(0.0, w * 1024.0));
    }
    for (int bit = 9; bit >= 0; --bit)
      for (int a = 2; a >= 0; --a) k = (k << 1) | ((q[a] >> bit) & 1u);
    key[e] = (int64_t)k * E + e;   // ties broken by the element index
  }
  std::vector<int> idx(E);
  for (int e = 0; e < E; ++e) idx[e] = e;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return key[x] < key[y]; });
  std::vector<int64_t> rank(E);
  for (int r = 0; r < E; ++r) rank[idx[r]] = r;
  return rank;
}

// Local refinement (Sec. 3.1): `steps` levels above the finest spec (the base).  On each level
// the listed active elements are refined regularly (8 active children) and the other elements
// of their 3 x 3 x 3 blocks irregularly (8 frozen children); a marked element's in-domain block
// must be active.  Children follow their parents in id order, child c = bx + 2 by + 4 bz, with
// the parent's map evaluated at the child's nodes.  A child face lies inside its parent (a
// sibling), on a parent face toward a refined neighbour (that neighbour's child across the
// face), on the domain boundary (the parent's code) or toward an unrefined element
// (kLevelEdge: frozen children only).
template <class SpecT>
void add_local_specs(std::vector<SpecT>& sp, const dgfas_mesh_desc* m, int steps) {
  SpecT& B = sp.back();
  const int p = B.deg[0], n = p + 1, n3 = n * n * n;
  B.X.assign(m->coords, m->coords + (size_t)B.E * 3 * n3);
  B.cls.assign(B.E, kLeaf);
  const std::vector<double> Mh = h_child_matrices(p);   // [6][n][n]: P0, P1, I0^T, I1^T, I0, I1
  const double* Ib[2] = {&Mh[(size_t)4 * n * n], &Mh[(size_t)5 * n * n]};
  int64_t pos = 0;
  for (int k = 0; k < steps; ++k) {
    SpecT& P = sp.back();
    const int E = P.E;
    auto walk = [&](int e, const int dd[3], bool& edge) {
      int cur = e;
      edge = false;
      for (int d = 0; d < 3 && cur >= 0; ++d)
        if (dd[d]) {
          const int f = 2 * d + (dd[d] > 0);
          const int nx = P.nbr[(size_t)cur * 6 + f];
          if (nx < 0 && P.bc[(size_t)cur * 6 + f] == kLevelEdge) edge = true;
          cur = nx;
        }
      return cur;
    };
    std::vector<int8_t> kind(E, -1);   // kTwig: regular, kFrozen: irregular
    const int cnt = m->refine_count[k];
    if (cnt < 0) throw Error(DGFAS_EINVAL, "negative refine_count");
    for (int q = 0; q < cnt; ++q) {
      const int e = m->refine_list[pos + q];
      if (e < 0 || e >= E) throw Error(DGFAS_EINVAL, "refine_list entry out of range");
      if (P.cls[e] == kFrozen) throw Error(DGFAS_EINVAL, "a frozen element cannot be refined");
      if (kind[e] == kTwig) throw Error(DGFAS_EINVAL, "an element is listed twice for refinement");
      kind[e] = kTwig;
    }
    for (int q = 0; q < cnt; ++q) {
      const int e = m->refine_list[pos + q];
      for (int d3 = -1; d3 <= 1; ++d3)
        for (int d2 = -1; d2 <= 1; ++d2)
          for (int d1 = -1; d1 <= 1; ++d1) {
            const int dd[3] = {d1, d2, d3};
            bool edge = false;
            const int x = walk(e, dd, edge);
            if (edge || (x >= 0 && P.cls[x] == kFrozen))
              throw Error(DGFAS_EINVAL, "a refined element needs an active 3 x 3 x 3 block inside the domain");
            if (x >= 0 && kind[x] != kTwig) kind[x] = kFrozen;
          }
    }
    pos += cnt;
    SpecT C;
    C.E = 0;
    C.hdown = false;
    C.box[0] = C.box[1] = C.box[2] = 0;
    std::vector<int> first(E, -1);
    for (int e = 0; e < E; ++e)
      if (kind[e] >= 0) {
        first[e] = C.E;
        C.E += 8;
        (kind[e] == kTwig ? C.tw : C.ir).push_back(e);
      }
    if (C.E == 0) throw Error(DGFAS_EINVAL, "a refinement step refines no element");
    C.deg.assign(C.E, p);
    C.nbr.assign((size_t)C.E * 6, -1);
    C.bc.assign((size_t)C.E * 6, DGFAS_INTERIOR);
    C.cls.assign(C.E, kLeaf);
    C.X.assign((size_t)C.E * 3 * n3, 0.0);
    std::vector<double> t1(n3), t2(n3);
    for (int e = 0; e < E; ++e) {
      if (kind[e] < 0) continue;
      if (kind[e] == kTwig) P.cls[e] = kTwig;
      for (int c = 0; c < 8; ++c) {
        const int ch = first[e] + c;
        const int b[3] = {c & 1, (c >> 1) & 1, c >> 2};
        C.cls[ch] = kind[e] == kTwig ? kLeaf : kFrozen;
        (kind[e] == kTwig ? C.twc : C.irc).push_back(ch);
        for (int a = 0; a < 3; ++a) {   // X_child = (I_bz x I_by x I_bx) X_parent
          const double* xp = &P.X[((size_t)e * 3 + a) * n3];
          for (int kk = 0; kk < n; ++kk)
            for (int j = 0; j < n; ++j)
              for (int i = 0; i < n; ++i) {
                double v = 0;
                for (int q = 0; q < n; ++q) v += Ib[b[0]][i * n + q] * xp[(kk * n + j) * n + q];
                t1[(kk * n + j) * n + i] = v;
              }
          for (int kk = 0; kk < n; ++kk)
            for (int j = 0; j < n; ++j)
              for (int i = 0; i < n; ++i) {
                double v = 0;
                for (int q = 0; q < n; ++q) v += Ib[b[1]][j * n + q] * t1[(kk * n + q) * n + i];
                t2[(kk * n + j) * n + i] = v;
              }
          double* xc = &C.X[((size_t)ch * 3 + a) * n3];
          for (int kk = 0; kk < n; ++kk)
            for (int j = 0; j < n; ++j)
              for (int i = 0; i < n; ++i) {
                double v = 0;
                for (int q = 0; q < n; ++q) v += Ib[b[2]][kk * n + q] * t2[(q * n + j) * n + i];
                xc[(kk * n + j) * n + i] = v;
              }
        }
        for (int f = 0; f < 6; ++f) {
          const int ax = f >> 1, sd = f & 1;
          if (b[ax] != sd) {   // the sibling across the parent's mid-plane
            C.nbr[(size_t)ch * 6 + f] = first[e] + (c ^ (1 << ax));
            continue;
          }
          const int en = P.nbr[(size_t)e * 6 + f];
          if (en < 0) {
            C.bc[(size_t)ch * 6 + f] = P.bc[(size_t)e * 6 + f];
          } else if (kind[en] >= 0) {
            C.nbr[(size_t)ch * 6 + f] = first[en] + (c ^ (1 << ax));
          } else {
            if (kind[e] == kTwig) throw Error(DGFAS_EINVAL, "an active child without its neighbour");
            C.bc[(size_t)ch * 6 + f] = kLevelEdge;
          }
        }
      }
    }
    sp.push_back(std::move(C));
  }
}

Solver* create(const dgfas_mesh_desc* m, const dgfas_options* o, void* stream) {
  validate(m, o);
  std::unique_ptr<Solver> s(new Solver());
  HIPC(hipGetDevice(&s->dev));
  {
    int cus = 0;
    HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->dev));
    s->cus = std::max(1, cus);
  }
  resolve_scratch(s->dev);
  if (o->null_space) s->npart = s->own(dalloc<double>((size_t)1024 * std::max(1, o->n_rhs)));
  s->opt = *o;
  s->st = (hipStream_t)stream;
  s->E = m->n_elem;
  const int E = s->E;
  s->h_nbr.assign(m->face_nbr, m->face_nbr + (size_t)E * 6);
  s->h_bc.assign(m->face_bc, m->face_bc + (size_t)E * 6);
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f)
      if (s->h_nbr[e * 6 + f] >= 0) s->h_bc[e * 6 + f] = DGFAS_INTERIOR;
  s->nbr = s->own(upload(s->h_nbr, s->st));
  s->bc = s->own(upload(s->h_bc, s->st));
  s->nrhs = o->n_rhs;
  if (o->order == DGFAS_ORDER_MORTON) s->rank = morton_rank(m);
  s->reserve(s->partial, (size_t)2048 * s->nrhs);
  s->reserve(s->scal, (size_t)8 * s->nrhs);
  s->reserve(s->dotout, (size_t)8 * s->nrhs);
  // face tables of the mixed-degree kernel: D of degrees 1..8 (stride 81) and the
  // interpolation from degree q to degree r at ((q - 1) 8 + r - 1) 81
  {
    std::vector<double> Dall(8 * 81, 0.0), Iall(64 * 81, 0.0);
    for (int q = 1; q <= 8; ++q) {
      const Gll& g = gll_table(q);
      for (size_t i = 0; i < g.D.size(); ++i) Dall[(q - 1) * 81 + i] = g.D[i];
      for (int r = 1; r <= 8; ++r) {
        std::vector<double> I = interp_matrix(q, r);
        for (size_t i = 0; i < I.size(); ++i) Iall[((q - 1) * 8 + (r - 1)) * 81 + i] = I[i];
      }
    }
    s->Dall = s->own(upload(Dall, s->st));
    s->Iall = s->own(upload(Iall, s->st));
  }
  // Level specs, finest first: h_levels h-coarsenings at the fine degree (Sec. 3.1: 2 x 2 x 2
  // children per parent), then, unless h_only, the per-element degree chain
  // p_{l-1} = max(1, floor(p_l / 2)) on the coarsest h-mesh
  struct Spec {
    int E;
    std::vector<int> deg, nbr;
    std::vector<int8_t> bc;
    int box[3];
    bool hdown;
    std::vector<int> children;   // [E of the next coarser spec][8] when hdown
    // local refinement: classes, host coordinates, and the transfer lists to the spec below
    std::vector<int8_t> cls;
    std::vector<double> X;
    std::vector<int> tw, twc, ir, irc;
  };
  std::vector<Spec> sp;
  sp.push_back({E, std::vector<int>(m->degree, m->degree + E), s->h_nbr, s->h_bc, {m->box[0], m->box[1], m->box[2]},
                false, {}});
  for (int h = 0; h < o->h_levels; ++h) {
    Spec& F = sp.back();
    const int nx = F.box[0], ny = F.box[1], NX = nx / 2, NY = F.box[1] / 2, NZ = F.box[2] / 2;
    const int Ec = NX * NY * NZ;
    Spec C{Ec, std::vector<int>(Ec, F.deg[0]), std::vector<int>((size_t)Ec * 6, -1),
           std::vector<int8_t>((size_t)Ec * 6, DGFAS_INTERIOR), {NX, NY, NZ}, false, {}};
    F.children.resize((size_t)Ec * 8);
    for (int P = 0; P < Ec; ++P) {
      const int Px = P % NX, Py = (P / NX) % NY, Pz = P / (NX * NY);
      for (int c = 0; c < 8; ++c)
        F.children[(size_t)P * 8 + c] = (2 * Px + (c & 1)) + nx * ((2 * Py + ((c >> 1) & 1)) + ny * (2 * Pz + (c >> 2)));
      // a parent face takes its neighbour and boundary code from a child on that face
      for (int f = 0; f < 6; ++f) {
        const int ch = F.children[(size_t)P * 8 + ((f & 1) << (f >> 1))];
        const int en = F.nbr[(size_t)ch * 6 + f];
        if (en >= 0) {
          const int ex = en % nx, ey = (en / nx) % ny, ez = en / (nx * ny);
          C.nbr[(size_t)P * 6 + f] = ex / 2 + NX * (ey / 2 + NY * (ez / 2));
        } else {
          C.bc[(size_t)P * 6 + f] = F.bc[(size_t)ch * 6 + f];
        }
      }
    }
    F.hdown = true;
    sp.push_back(std::move(C));
  }
  if (!o->h_only) {
    while (*std::max_element(sp.back().deg.begin(), sp.back().deg.end()) > 1) {
      Spec C = sp.back();
      C.hdown = false;
      C.children.clear();
      for (int& d : C.deg) d = std::max(1, d / 2);
      sp.push_back(std::move(C));
    }
  }
  std::reverse(sp.begin(), sp.end());   // root first
  if (o->local_steps > 0) add_local_specs(sp, m, o->local_steps);
  const int Lc = (int)sp.size();
  s->lv.resize(Lc);
  for (int li = 0; li < Lc; ++li) {
    Level& L = s->lv[li];
    L.E = sp[li].E;
    L.h_nbr = sp[li].nbr;
    L.h_bc = sp[li].bc;
    for (int8_t& c : L.h_bc)   // a frozen element's face toward the unrefined region: no face term
      if (c == kLevelEdge) c = DGFAS_NEUMANN;
    L.lr = !sp[li].cls.empty();
    L.h_cls = sp[li].cls;
    if (!sp[li].tw.empty() || !sp[li].ir.empty()) {
      L.lr_down = true;
      L.ntw = (int)sp[li].tw.size();
      L.nir = (int)sp[li].ir.size();
      if (L.ntw) { L.tw_par = s->own(upload(sp[li].tw, s->st)); L.tw_ch = s->own(upload(sp[li].twc, s->st)); }
      if (L.nir) { L.ir_par = s->own(upload(sp[li].ir, s->st)); L.ir_ch = s->own(upload(sp[li].irc, s->st)); }
      L.hM = s->own(upload(h_child_matrices(sp[li].deg[0]), s->st));
    }
    for (int d = 0; d < 3; ++d) L.box[d] = sp[li].box[d];
    if (m->face_nbr_face) {
      // p-levels keep the topology: every level has the mesh's faces and orientations
      L.topo = true;
      L.h_nface.assign(m->face_nbr_face, m->face_nbr_face + (size_t)E * 6);
      L.h_norient.assign((size_t)E * 6, 0);
      if (m->face_orient) L.h_norient.assign(m->face_orient, m->face_orient + (size_t)E * 6);
      std::vector<int8_t> pk((size_t)E * 6, 0);
      for (size_t q = 0; q < pk.size(); ++q)
        if (L.h_nbr[q] >= 0) pk[q] = (int8_t)(L.h_nface[q] | (L.h_norient[q] << 3));
      L.nfo = s->own(upload(pk, s->st));
    }
    L.nbr = s->own(upload(L.h_nbr, s->st));
    L.bc = s->own(upload(L.h_bc, s->st));
    L.hdown = sp[li].hdown;
    if (L.hdown) {
      L.hchild = s->own(upload(sp[li].children, s->st));
      L.hM = s->own(upload(h_child_matrices(sp[li].deg[0]), s->st));
    }
  }
  auto ncoords = [](const std::vector<int>& dg) {
    size_t n = 0;
    for (int d : dg) n += (size_t)3 * (d + 1) * (d + 1) * (d + 1);
    return n;
  };
  // the finest level's coordinates: the mesh's, or those of the top locally refined level
  double* X = s->own(dalloc<double>(ncoords(sp[Lc - 1].deg)));
  HIPC(hipMemcpyAsync(X, sp[Lc - 1].X.empty() ? m->coords : sp[Lc - 1].X.data(),
                      ncoords(sp[Lc - 1].deg) * sizeof(double), hipMemcpyHostToDevice, s->st));
  // a nodal diffusivity follows the geometry from level to level (one component)
  double* NU = nullptr;
  if (m->nu_nodal) {
    NU = s->own(dalloc<double>(ncoords(sp[Lc - 1].deg) / 3));
    HIPC(hipMemcpyAsync(NU, m->nu_nodal, ncoords(sp[Lc - 1].deg) / 3 * sizeof(double), hipMemcpyHostToDevice,
                        s->st));
  }
  for (int li = Lc - 1; li >= 0; --li) {
    Level& L = s->lv[li];
    const std::vector<int>& dgl = sp[li].deg;
    if (li < Lc - 1 && !sp[li].X.empty()) {
      // a locally refined level or its base: coordinates built on the host
      X = s->own(dalloc<double>(ncoords(dgl)));
      HIPC(hipMemcpyAsync(X, sp[li].X.data(), ncoords(dgl) * sizeof(double), hipMemcpyHostToDevice, s->st));
    } else if (li < Lc - 1) {
      // coarse geometry: the fine map evaluated at the coarse GLL nodes, per element (p) or per
      // parent from its children (h, averaged where the children meet)
      Level& F = s->lv[li + 1];
      double* Xc = s->own(dalloc<double>(ncoords(dgl)));
      double* NUc = NU ? s->own(dalloc<double>(ncoords(dgl) / 3)) : nullptr;
      if (F.hdown) {
        HXferArgs<double> a;
        a.kind = 0; a.ncoarse = L.E; a.children = F.hchild; a.ncomp = 3; a.M = F.hM; a.in = X; a.out = Xc;
        if (!htransfer<double>(F.p, a, s->st)) throw Error(DGFAS_EUNSUPPORTED, "no h-transfer kernel for this degree");
        HIPC(hipGetLastError());
        if (NU) {
          a.ncomp = 1; a.in = NU; a.out = NUc;
          htransfer<double>(F.p, a, s->st);
          HIPC(hipGetLastError());
        }
      } else {
        const int Ep = L.E;
        std::vector<int64_t> offc(Ep);
        int64_t oc = 0;
        for (int e = 0; e < Ep; ++e) { offc[e] = oc; oc += (int64_t)(dgl[e] + 1) * (dgl[e] + 1) * (dgl[e] + 1); }
        int64_t* d_offc = F.uniform ? nullptr : s->own(upload(offc, s->st));
        const bool cu = *std::min_element(dgl.begin(), dgl.end()) == *std::max_element(dgl.begin(), dgl.end());
        for (Bucket& b : F.bk) {
          const int pf = b.p, pc = std::max(1, pf / 2);
          // the geometry of the coarse level is the fine map evaluated at the coarse nodes; the
          // solution projection is that evaluation or the L2 projection (Sec. 3.2)
          std::vector<double> Pg = interp_matrix(pf, pc), I = interp_matrix(pc, pf);
          std::vector<double> P = s->opt.projection == DGFAS_PROJECT_L2 && pc < pf ? l2_projection_matrix(pf, pc) : Pg;
          std::vector<double> R((size_t)(pc + 1) * (pf + 1));
          for (int a = 0; a <= pc; ++a)
            for (int c = 0; c <= pf; ++c) R[a * (pf + 1) + c] = I[c * (pc + 1) + a];
          b.pc = pc;
          b.Pm = s->own(upload(P, s->st));
          b.Im = s->own(upload(I, s->st));
          b.Rm = s->own(upload(R, s->st));
          double* Pgeo = s->own(upload(Pg, s->st));
          XferArgs<double> a;
          a.Tm = Pgeo; a.in = X; a.out = Xc;
          if (F.uniform) {
            a.nel = 3 * Ep;
          } else {
            a.nel = b.nel; a.elist = b.elist; a.ncomp = 3; a.off_in = F.off; a.off_out = cu ? nullptr : d_offc;
          }
          if (!tensor3<double>(pf + 1, pc + 1, a, s->st))
            throw Error(DGFAS_EUNSUPPORTED, "no transfer kernel for this degree pair");
          HIPC(hipGetLastError());
          if (NU) {   // one degree: the whole level is one block of E elements
            XferArgs<double> an;
            an.Tm = Pgeo; an.in = NU; an.out = NUc; an.nel = Ep;
            tensor3<double>(pf + 1, pc + 1, an, s->st);
            HIPC(hipGetLastError());
          }
        }
      }
      X = Xc;
      NU = NUc;
    }
    build_level(*s, L, dgl, X, NU);
    L.X = X;
    if (li < Lc - 1) {
      s->reserve(L.u, (size_t)L.ndof * s->nrhs, L.lr);
      s->reserve(L.g, (size_t)L.ndof * s->nrhs, L.lr);
      s->reserve(L.ubar, (size_t)L.ndof * s->nrhs, L.lr);
    }
  }
  // the workspace: one library-owned block until the caller hands in its own buffer
  s->ws_bytes = s->ws_layout();
  s->ws_block = dalloc<char>(s->ws_bytes);
  s->ws_assign(static_cast<char*>(s->ws_block));
  HIPC(hipStreamSynchronize(s->st));
  return s.release();
}

}  // namespace

const char* set_error(const std::string& m) {
  g_err = m;
  return g_err.c_str();
}

namespace {

dgfas_status fail(const Error& e) {
  g_err = e.what();
  return e.code;
}

}  // namespace
}  // namespace dgfas

using namespace dgfas;

struct dgfas_solver_s {
  Solver* s;
};

#define API_BEGIN try {
#define API_END                                           \
  }                                                       \
  catch (const Error& e) { return fail(e); }              \
  catch (const std::exception& e) {                       \
    g_err = e.what();                                     \
    return DGFAS_EINVAL;                                  \
  }                                                       \
  return DGFAS_OK;

static Solver* S_(dgfas_solver s) {
  if (!s || !s->s) throw Error(DGFAS_EINVAL, "null solver");
  return s->s;
}
static void need(const void* p, const char* what) {
  if (!p) throw Error(DGFAS_EINVAL, std::string("null pointer: ") + what);
}

extern "C" {

void dgfas_default_options(dgfas_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->kappa = 0.0;
  o->nu = 1.0;
  o->mu_star = 2.0;
  o->overlap = 1;
  o->smoother = DGFAS_WAS;
  o->ns1 = 2;
  o->ns2 = 2;
  o->root_max_iter = 500;
  o->root_rtol = 1e-12;
  o->precision = DGFAS_FP64;
  o->n_rhs = 1;
  o->start = DGFAS_START_NONE;
  o->weighting = DGFAS_WEIGHT_QUINTIC;
  o->delta = 0.08;
}

dgfas_status dgfas_gll(int32_t p, double* x, double* w) {
  API_BEGIN
  need(x, "x");
  need(w, "w");
  if (p < 1 || p > kMaxDegree) throw Error(DGFAS_EINVAL, "degree out of range");
  const Gll& g = gll_table(p);
  for (int i = 0; i <= p; ++i) { x[i] = g.x[i]; w[i] = g.w[i]; }
  API_END
}

dgfas_status dgfas_schwarz_tables_1d(int32_t p, int32_t m, int32_t left, int32_t right, double mu_star, int32_t* ns,
                                     double* S, double* lam, double* weights) {
  API_BEGIN
  need(ns, "ns"); need(S, "S"); need(lam, "lam"); need(weights, "weights");
  if (p < 1 || p > kMaxDegree || m < 0 || m > p) throw Error(DGFAS_EINVAL, "p or m out of range");
  if (left < 0 || left > 3 || right < 0 || right > 3) throw Error(DGFAS_EINVAL, "bad side code");
  Variant1D v = make_variant_1d(p, m, left, right, mu_star);
  *ns = v.ns;
  for (int i = 0; i < v.ns * v.ns; ++i) S[i] = v.S[i];
  for (int i = 0; i < v.ns; ++i) { lam[i] = v.lam[i]; weights[i] = v.W[i]; }
  API_END
}

dgfas_status dgfas_create(const dgfas_mesh_desc* mesh, const dgfas_options* opt, void* stream, dgfas_solver* out) {
  API_BEGIN
  need(out, "out");
  *out = nullptr;
  Solver* s = create(mesh, opt, stream);
  *out = new dgfas_solver_s{s};
  API_END
}

void dgfas_destroy(dgfas_solver s) {
  if (!s) return;
  delete s->s;
  delete s;
}

dgfas_status dgfas_levels(dgfas_solver s, int32_t* n) {
  API_BEGIN
  need(n, "n_levels");
  *n = (int32_t)S_(s)->lv.size();
  API_END
}

dgfas_status dgfas_level_info(dgfas_solver s, int32_t level, int32_t* degree, int64_t* n_dof) {
  API_BEGIN
  Level& L = S_(s)->level(level);
  if (degree) *degree = L.p;
  if (n_dof) *n_dof = L.ndof;
  API_END
}

dgfas_status dgfas_workspace_size(dgfas_solver sv, size_t* bytes) {
  API_BEGIN
  need(bytes, "bytes");
  *bytes = S_(sv)->ws_bytes;
  API_END
}

dgfas_status dgfas_set_workspace(dgfas_solver sv, void* dptr, size_t bytes) {
  API_BEGIN
  Solver* s = S_(sv);
  if (dptr) {
    if (bytes < s->ws_bytes)
      throw Error(DGFAS_EINVAL, "workspace of " + std::to_string(bytes) + " bytes, " +
                                    std::to_string(s->ws_bytes) + " needed");
    if (reinterpret_cast<uintptr_t>(dptr) % 256) throw Error(DGFAS_EINVAL, "workspace must be 256-byte aligned");
  }
  HIPC(hipStreamSynchronize(s->st));   // work still queued may use the current buffers
  s->drop_graphs();
  void* old = s->ws_block;
  if (dptr) {
    s->ws_assign(static_cast<char*>(dptr));
    s->ws_block = nullptr;
  } else {
    void* blk = dalloc<char>(s->ws_bytes);
    s->ws_assign(static_cast<char*>(blk));
    s->ws_block = blk;
  }
  HIPC(hipStreamSynchronize(s->st));
  if (old && old != s->ws_block) HIPC(hipFree(old));
  API_END
}

dgfas_status dgfas_level_overlap(dgfas_solver s, int32_t level, int32_t* m) {
  API_BEGIN
  need(m, "m");
  *m = S_(s)->level(level).m;
  API_END
}

dgfas_status dgfas_level_blocks(dgfas_solver s, int32_t level, int64_t* counts) {
  API_BEGIN
  need(counts, "counts");
  const Level& L = S_(s)->level(level);
  for (int k = 0; k < 5; ++k) counts[k] = L.tblocks[k];
  API_END
}

namespace dgfas {
namespace {
void level_rhs(Solver* s, Level& T, const double* f, const double* uD, const double* qN, double* b) {
  for (int k = 0; k < s->nrhs; ++k) {
    const int64_t o = (int64_t)k * T.ndof;
    for (const Bucket& bk : T.bk) {
      RhsArgs a;
      a.nel = bk.nel; a.elist = bk.elist; a.off = T.off; a.offF = T.offF; a.ndof = T.ndof;
      a.f = f + o; a.uD = uD ? uD + o : nullptr; a.qN = qN ? qN + o : nullptr; a.b = b + o;
      a.G = T.G; a.WJ = T.WJ; a.pen = T.pen; a.ws = T.ws; a.nbr = T.nbr; a.bc = T.bc;
      rhs(bk.p, a, bk.t->D, bk.t->inv_wend, s->st);
    }
  }
  HIPC(hipGetLastError());
}
}  // namespace
}  // namespace dgfas

dgfas_status dgfas_rhs(dgfas_solver sv, const double* f, const double* uD, const double* qN, double* b) {
  API_BEGIN
  Solver* s = S_(sv);
  need(f, "f"); need(b, "b");
  level_rhs(s, s->lv.back(), f, uD, qN, b);
  API_END
}

dgfas_status dgfas_level_rhs(dgfas_solver sv, int32_t level, const double* f, const double* uD, const double* qN,
                             double* b) {
  API_BEGIN
  Solver* s = S_(sv);
  need(f, "f"); need(b, "b");
  level_rhs(s, s->level(level), f, uD, qN, b);
  API_END
}

dgfas_status dgfas_level_classes(dgfas_solver sv, int32_t level, int8_t* cls) {
  API_BEGIN
  Solver* s = S_(sv);
  need(cls, "cls");
  Level& L = s->level(level);
  for (int e = 0; e < L.E; ++e) cls[e] = L.lr ? L.h_cls[e] : kTwig + (level == (int)s->lv.size() ? kLeaf : 0);
  API_END
}

dgfas_status dgfas_level_coords(dgfas_solver sv, int32_t level, double* coords) {
  API_BEGIN
  Solver* s = S_(sv);
  need(coords, "coords");
  Level& L = s->level(level);
  HIPC(hipMemcpyAsync(coords, L.X, (size_t)3 * L.ndof * sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPC(hipStreamSynchronize(s->st));
  API_END
}

dgfas_status dgfas_set_level_rhs(dgfas_solver sv, int32_t level, const double* b) {
  API_BEGIN
  Solver* s = S_(sv);
  need(b, "b");
  if (level == (int)s->lv.size()) throw Error(DGFAS_EINVAL, "the top level's right-hand side is the solve's f");
  if (s->opt.local_steps <= 0) throw Error(DGFAS_EINVAL, "per-level right-hand sides need local refinement");
  Level& L = s->level(level);
  if (!L.bfull) L.bfull = s->own(dalloc<double>(L.ndof));
  HIPC(hipMemcpyAsync(L.bfull, b, (size_t)L.ndof * sizeof(double), hipMemcpyDeviceToDevice, s->st));
  API_END
}

dgfas_status dgfas_level_solution(dgfas_solver sv, int32_t level, double* u) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u");
  if (level == (int)s->lv.size()) throw Error(DGFAS_EINVAL, "the top level's solution is the solve's u");
  Level& L = s->level(level);
  HIPC(hipMemcpyAsync(u, L.u, (size_t)L.ndof * sizeof(double), hipMemcpyDeviceToDevice, s->st));
  API_END
}

dgfas_status dgfas_apply(dgfas_solver sv, int32_t level, const double* u, double* Au) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(Au, "Au");
  s->apply(s->level(level), u, Au);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_residual(dgfas_solver sv, int32_t level, const double* u, const double* g, double* r) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(g, "g"); need(r, "r");
  s->residual(s->level(level), u, g, r);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_schwarz(dgfas_solver sv, int32_t level, const double* r, double* z) {
  API_BEGIN
  Solver* s = S_(sv);
  need(r, "r"); need(z, "z");
  s->schwarz(s->level(level), r, z, 0);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_schwarz_noalloc(dgfas_solver sv, int32_t level, const double* r, double* z) {
  API_BEGIN
  Solver* s = S_(sv);
  need(r, "r"); need(z, "z");
  Level& L = s->level(level);
  if (L.topo)
    throw Error(DGFAS_EUNSUPPORTED, "the allocation-free Schwarz application covers structured meshes only");
  const size_t need_d = (size_t)L.nin * s->nrhs;
  if (need_d > kNoAllocDoubles)
    throw Error(DGFAS_EINVAL, "level " + std::to_string(level) + " needs an overlap inbox of " +
                                  std::to_string(need_d) + " doubles, more than the " +
                                  std::to_string(kNoAllocDoubles) + " of the static scratch array");
  if (s->learned && &L == &s->lv.back())
    throw Error(DGFAS_EUNSUPPORTED, "the learned correction's network may allocate; detach it first");
  double* box = scratch_address(s->dev);
  if (!box) throw Error(DGFAS_EHIP, "scratch array not resolved on this device");
  struct Reset {   // the override never outlives the call, also when it throws
    Solver* s;
    ~Reset() { s->inbox64 = nullptr; }
  } reset{s};
  // regions that no subdomain writes (absent neighbours, another degree) must read zero, and the
  // array holds whatever the last call on this device left in it
  if (need_d) fill((int64_t)need_d, box, 0.0, s->st);
  s->inbox64 = box;
  s->schwarz(L, r, z, 0);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_smooth(dgfas_solver sv, int32_t level, double* u, const double* g, int32_t n) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(g, "g");
  if (n < 0) throw Error(DGFAS_EINVAL, "negative step count");
  s->smooth(s->level(level), u, g, n);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_restrict(dgfas_solver sv, int32_t level, const double* rf, double* rc) {
  API_BEGIN
  Solver* s = S_(sv);
  need(rf, "r_fine"); need(rc, "r_coarse");
  if (level < 2) throw Error(DGFAS_EINVAL, "restrict needs level >= 2");
  Level& F = s->level(level);
  Level& C = s->level(level - 1);
  s->transfer(F, C, 1, rf, nullptr, rc, 0);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_project(dgfas_solver sv, int32_t level, const double* uf, double* uc) {
  API_BEGIN
  Solver* s = S_(sv);
  need(uf, "u_fine"); need(uc, "u_coarse");
  if (level < 2) throw Error(DGFAS_EINVAL, "project needs level >= 2");
  Level& F = s->level(level);
  Level& C = s->level(level - 1);
  s->transfer(F, C, 0, uf, nullptr, uc, 0);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_prolong_add(dgfas_solver sv, int32_t level, const double* uc, const double* ubar, double* uf) {
  API_BEGIN
  Solver* s = S_(sv);
  need(uc, "u_coarse"); need(uf, "u_fine");
  if (level < 2) throw Error(DGFAS_EINVAL, "prolong needs level >= 2");
  Level& F = s->level(level);
  Level& C = s->level(level - 1);
  s->transfer(F, C, 2, uc, ubar, uf, 1);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_root_solve(dgfas_solver sv, double* u, const double* g, int32_t* iters) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(g, "g");
  bool bd = false;
  const int it = s->root_solve(u, g, &bd);
  HIPC(hipStreamSynchronize(s->st));
  if (iters) *iters = it;
  if (bd) throw Error(DGFAS_EBREAKDOWN, "SCG breakdown in the root solve");
  API_END
}

dgfas_status dgfas_startup(dgfas_solver sv, double* u, const double* f) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(f, "f");
  s->startup(u, f);
  HIPC(hipStreamSynchronize(s->st));
  API_END
}

dgfas_status dgfas_vcycle(dgfas_solver sv, double* u, const double* f) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(f, "f");
  s->vcycle(u, f);
  HIPC(hipGetLastError());
  API_END
}

dgfas_status dgfas_solve(dgfas_solver sv, double* u, const double* f, int32_t max_cycles, double rtol, double* hist,
                         int32_t* n_done) {
  API_BEGIN
  Solver* s = S_(sv);
  need(u, "u"); need(f, "f");
  if (max_cycles < 0) throw Error(DGFAS_EINVAL, "negative max_cycles");
  struct HintReset {   // no residual hint or crossover count survives the call, also when it throws
    Solver* s;
    ~HintReset() {
      s->rhint = false;
      s->ns1_top = -1;
    }
  } hint_reset{s};
  Level& T = s->lv.back();
  if (s->opt.local_steps > 0) {
    // local refinement: the lower levels start from zero, and the history is that of the
    // composite residual over the leaves of every level
    for (size_t l = 0; l + 1 < s->lv.size(); ++l) {
      Level& L = s->lv[l];
      fill(L.ndof, L.u, 0.0, s->st);
      if (L.lr && L.nleaf) {
        if (!L.bfull) throw Error(DGFAS_EINVAL, "a level with leaves has no right-hand side (dgfas_set_level_rhs)");
        copy_rows(L.leaf_list, L.nleaf, L.N3, L.bfull, L.g, s->st);
      }
    }
    s->rhint = false;
    const double r0 = std::sqrt(s->composite_norm2(u, f));
    if (s->opt.start == DGFAS_START_FMG) {
      for (size_t l = 0; l + 1 < s->lv.size(); ++l)
        if (!s->lv[l].bfull) throw Error(DGFAS_EINVAL, "the FMG start-up needs every level's right-hand side");
      s->startup_lr(u);
    }
    if (hist) hist[0] = 1.0;
    int k = 0;
    bool conv = r0 == 0.0;
    while (!conv && k < max_cycles) {
      s->vcycle(u, f);
      const double rk = std::sqrt(s->composite_norm2(u, f)) / r0;
      ++k;
      if (hist) hist[k] = rk;
      if (!std::isfinite(rk)) throw Error(DGFAS_EBREAKDOWN, "non-finite residual");
      conv = rk <= rtol;
    }
    if (n_done) *n_done = k;
    if (!conv) { g_err = "tolerance not reached"; return DGFAS_ENOTCONV; }
    return DGFAS_OK;
  }
  s->residual(T, u, f, T.r);
  std::vector<double> r0 = s->dots_sync(T, T.r, T.r);
  for (double& v : r0) v = std::sqrt(v);
  if (s->opt.start != DGFAS_START_NONE) {
    s->startup(u, f);
    s->residual(T, u, f, T.r);   // the cycles below take T.r as f - A u of the start value
  }
  // crossover: every cycle after the first starts with nsc - ns2 finest-level pre-smoothing steps
  const int nsc = s->opt.nsc > 0 ? s->opt.nsc : s->opt.ns1 + s->opt.ns2;
  const int pre_later = nsc - s->opt.ns2;
  const bool crossover = pre_later != s->opt.ns1;
  if (hist) hist[0] = 1.0;
  int k = 0;
  auto worst = [&](const std::vector<double>& rr) {
    double w = 0.0;
    for (int j = 0; j < s->nrhs; ++j) {
      const double rel = r0[j] > 0.0 ? std::sqrt(rr[j]) / r0[j] : 0.0;
      if (!std::isfinite(rel)) return rel;
      w = std::max(w, rel);
    }
    return w;
  };
  bool conv = worst(std::vector<double>(s->nrhs, 0.0)) == 0.0 &&
              *std::max_element(r0.begin(), r0.end()) == 0.0;
  // learned correction: the plain smoother is the judge.  The first solve after attaching runs
  // its first two cycles plain; the second cycle's reduction factor is the reference (the first
  // cycle of any solve reduces far more than later ones).  A learned cycle that reduces less than
  // the reference, or goes non-finite, is undone and the solve continues plain.
  const bool attached = s->learned;
  bool use_learned = attached, fell_back = false;
  if (attached && !s->usave) s->usave = s->own(dalloc<double>(T.ndof * s->nrhs));
  double* usave = s->usave;
  double prev = 1.0;
  while (!conv && k < max_cycles) {
    const bool plain_probe = use_learned && s->plain_rho < 0.0;
    s->learned = use_learned && !plain_probe;
    if (s->learned)
      HIPC(hipMemcpyAsync(usave, u, T.ndof * s->nrhs * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    s->rhint = true;   // T.r holds f - A u of this u (computed before the loop or below)
    s->ns1_top = (crossover && k > 0) ? pre_later : -1;
    // the first cycle of a crossover solve runs eagerly, so that the graphs keep the later cycles' shape
    if (s->opt.graph && !attached && !(crossover && k == 0)) s->vcycle_graphed(u, f);
    else s->vcycle(u, f);
    s->rhint = false;
    s->residual(T, u, f, T.r);
    double rk = worst(s->dots_sync(T, T.r, T.r));
    if (plain_probe && k == 1) s->plain_rho = rk / prev;
    if (s->learned && s->judge && (!std::isfinite(rk) || rk / prev > s->plain_rho)) {
      HIPC(hipMemcpyAsync(u, usave, T.ndof * s->nrhs * sizeof(double), hipMemcpyDeviceToDevice, s->st));
      use_learned = false;
      fell_back = true;
      s->learned = false;
      s->vcycle(u, f);
      s->residual(T, u, f, T.r);
      rk = worst(s->dots_sync(T, T.r, T.r));
    }
    ++k;
    if (hist) hist[k] = rk;
    if (!std::isfinite(rk)) { s->learned = attached; throw Error(DGFAS_EBREAKDOWN, "non-finite residual"); }
    prev = rk;
    conv = rk <= rtol;
  }
  s->learned = attached;
  if (n_done) *n_done = k;
  if (!conv) { g_err = "tolerance not reached"; return DGFAS_ENOTCONV; }
  if (fell_back) { g_err = "learned correction disabled by the fallback rule"; return DGFAS_EFALLBACK; }
  API_END
}


dgfas_status dgfas_norm(dgfas_solver sv, int32_t level, const double* v, double* out) {
  API_BEGIN
  Solver* s = S_(sv);
  need(v, "v"); need(out, "out");
  std::vector<double> d = s->dots_sync(s->level(level), v, v);
  for (int k = 0; k < s->nrhs; ++k) out[k] = std::sqrt(d[k]);
  API_END
}

dgfas_status dgfas_set_learned(dgfas_solver sv, dgfas_mlp m, int32_t enabled) {
  API_BEGIN
  Solver* s = S_(sv);
  Level& T = s->lv.back();
  if (!enabled) { s->learned = false; return DGFAS_OK; }
  if (s->opt.local_steps > 0) throw Error(DGFAS_EUNSUPPORTED, "no learned correction with local refinement");
  if (T.topo) throw Error(DGFAS_EUNSUPPORTED, "no learned correction on unstructured meshes");
  if (!m) throw Error(DGFAS_EINVAL, "null network");
  if (!T.uniform) throw Error(DGFAS_EUNSUPPORTED, "learned correction needs one degree on the finest level");
  Mlp* net = dgfas_mlp_impl(m);
  const int nt = T.ns * T.ns * T.ns;
  if (net->in != nt + 9 || net->out != nt)
    throw Error(DGFAS_EINVAL, "network shape must be (ns^3 + 9) -> ns^3 = " + std::to_string(nt + 9) + " -> " +
                                  std::to_string(nt));
  if (s->nrhs != 1) throw Error(DGFAS_EUNSUPPORTED, "learned correction needs n_rhs = 1");
  if (s->opt.precision != DGFAS_FP64) throw Error(DGFAS_EUNSUPPORTED, "learned correction runs in the FP64 smoother");
  if (!s->lX) {
    s->lX = s->own(dalloc<float>((size_t)T.E * (nt + 9)));
    s->lY = s->own(dalloc<float>((size_t)T.E * nt));
    s->lnorm = s->own(dalloc<double>(T.E));
  }
  net->st = s->st;
  s->mlp = net;
  s->learned = true;
  s->judge = enabled != 2;
  s->plain_rho = -1.0;
  API_END
}

dgfas_status dgfas_learned_pairs(dgfas_solver sv, const double* r, const int32_t* centers, int32_t n, float* X,
                                 float* T, int32_t* pcg_iters) {
  API_BEGIN
  Solver* s = S_(sv);
  need(r, "r"); need(centers, "centers"); need(X, "X"); need(T, "T");
  if (s->nrhs != 1) throw Error(DGFAS_EUNSUPPORTED, "pairs need n_rhs = 1");
  Level& L = s->lv.back();
  if (!L.uniform) throw Error(DGFAS_EUNSUPPORTED, "pairs need one degree on the finest level");
  if (L.topo) throw Error(DGFAS_EUNSUPPORTED, "pairs need a structured mesh");
  if (n < 1 || n > L.E) throw Error(DGFAS_EINVAL, "bad number of centres");
  // centres must be 4 apart in the 26-neighbourhood graph: their 3x3x3 patches then neither
  // overlap nor touch, so the masked operator is block diagonal over the subdomains
  std::vector<char> is_center(L.E, 0);
  for (int c = 0; c < n; ++c) {
    const int e0 = centers[c];
    if (e0 < 0 || e0 >= L.E) throw Error(DGFAS_EINVAL, "centre out of range");
    if (is_center[e0]) throw Error(DGFAS_EINVAL, "repeated centre");
    is_center[e0] = 1;
  }
  for (int c = 0; c < n; ++c) {
    const int e0 = centers[c];
    std::vector<int> front{e0}, seen{e0};
    for (int hop = 0; hop < 3; ++hop) {
      std::vector<int> nxt;
      for (int e : front)
        for (int q = 0; q < 27; ++q) {
          const int en = L.h_nb27[(size_t)e * 27 + q];
          if (en < 0 || std::find(seen.begin(), seen.end(), en) != seen.end()) continue;
          if (is_center[en]) throw Error(DGFAS_EINVAL, "centres closer than 4 elements");
          seen.push_back(en);
          nxt.push_back(en);
        }
      front.swap(nxt);
    }
  }
  std::vector<int> ids(centers, centers + n);
  std::vector<uint8_t> sel(L.E, 0);
  for (int e : ids) sel[e] = 1;
  int* d_ids = upload(ids, s->st);
  uint8_t* d_sel = upload(sel, s->st);
  double *mask = nullptr, *b = nullptr, *z0 = nullptr, *x = nullptr, *nrm = nullptr;
  auto cleanup = [&]() {
    s->msel = nullptr;
    s->mmask = nullptr;
    hipStreamSynchronize(s->st);
    void* ps[] = {d_ids, d_sel, mask, b, z0, x, nrm};
    for (void* p : ps)
      if (p) hipFree(p);
  };
  try {
    mask = dalloc<double>(L.ndof);
    b = dalloc<double>(L.ndof);
    z0 = dalloc<double>(L.ndof);
    x = dalloc<double>(L.ndof);
    nrm = dalloc<double>(n);
    SchwarzArgs<double> a = s->sz_args<double>(L, L.bk[0], r, z0, 0);
    fill(L.ndof, mask, 0.0, s->st);
    mark_subdomains<double>(L.p, L.m, a, d_ids, n, mask, s->st);
    convert<double, double>(L.ndof, r, b, 0, s->st);
    mask_mul(L.ndof, b, mask, s->st);
    s->msel = d_sel;
    s->mmask = mask;
    s->schwarz(L, b, z0, 0);                      // FD solutions of the local problems
    const double bn = std::sqrt(s->dots_sync(L, b, b)[0]);
    bool bd = false;
    const int it = s->scg<double>(L, x, b, 1000, {1e-11 * bn}, &bd, true);   // exact local solves
    if (bd) throw Error(DGFAS_EBREAKDOWN, "breakdown in the local solves");
    s->msel = nullptr;
    s->mmask = nullptr;
    tile_features<double>(L.p, L.m, a, d_ids, n, b, L.J9, X, nrm, s->st);
    tile_diff<double>(L.p, L.m, a, d_ids, n, x, z0, nrm, T, s->st);
    HIPC(hipGetLastError());
    if (pcg_iters) *pcg_iters = it;
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
  API_END
}

dgfas_status dgfas_autotune(dgfas_solver sv, const char* cache_path, int32_t reps, double* report) {
  API_BEGIN
  Solver* s = S_(sv);
  s->autotune(cache_path, reps, report);
  API_END
}

const char* dgfas_last_error(void) { return g_err.c_str(); }

}  // extern "C"
