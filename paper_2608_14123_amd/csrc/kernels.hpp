// Host-side launch interface of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgfas {

// face results of the faces between degrees, per side: the row term and the three lifting rows
// on that side's face grid (first, second layout), 81 values each
constexpr int kMortarFaceRes = 4 * 81;

template <typename T>
struct OpArgs {
  int E = 0;
  int nrhs = 1;               // vectors are [nrhs][ndof]
  int nel = 0;                // elements of this launch (the degree bucket)
  const int* elist = nullptr; // [nel] element ids of the bucket (null: 0..nel-1)
  const int64_t* off = nullptr;   // [E] first DOF of every element (null: e (p+1)^3)
  const int64_t* offF = nullptr;  // [E] first face-node slot of every element (null: 6 e (p+1)^2)
  const int* deg = nullptr;   // [E] degree of every element (null: all equal); faces to another
                              // degree are left to the mortar kernel
  int64_t ndof = 0;           // DOF per right-hand side (stride of G, WJ and of the batch)
  const T* u = nullptr;
  const T* g = nullptr;
  T* out = nullptr;
  int mode = 0;               // 0: out = g - A u, 1: out = A u
  const T* G = nullptr;       // [6][ndof]
  const T* WJ = nullptr;      // [ndof] or null when kappa = 0
  const T* pen = nullptr;     // [E][6][n^2]
  const int* nbr = nullptr;   // [E][6]
  const int8_t* bc = nullptr; // [E][6]
  const T* D = nullptr;       // [n][n]
  T kappa = 0;
  T inv_wend = 0;             // 1 / w_0 = p (p + 1) / 2
  double* dotp = nullptr;     // mode 1 only: per tile u^T (A u) partial sums, [nrhs][tiles]
  const int8_t* nfo = nullptr;   // [E][6] unstructured meshes: the neighbour's face | orientation
                                 // code << 3 per interior face (null: aligned neighbours)
  // mixed levels: the faces between degrees, computed beforehand by the mortar face kernel
  const int* fmapE = nullptr;    // [E][6] result slot of face phi, or -1 (null: no such faces)
  const T* fres = nullptr;       // [nrhs][2 nface][kMortarFaceRes] row and lifting terms per side
  int64_t fres_stride = 0;       // values per right-hand side
};

template <typename T>
void sipg_apply(int p, const OpArgs<T>& a, hipStream_t st);

// Batched launches of mixed-degree levels: one launch per sweep stage covers a work list of
// tiles over all degree buckets (largest degree first), one tile per workgroup, so the
// hardware dispatcher balances the load.  Per-bucket data lives in a device table; the
// per-call vectors come with the stage's argument block.
template <typename T>
struct BucketDesc {
  int p = 0, m = 0, nel = 0, pad0 = 0;
  int tile0[4] = {0, 0, 0, 0};      // first tile in the operator / solve / overlap-add lists
  const int* elist = nullptr;
  const T* D = nullptr;
  const T *S = nullptr, *ST = nullptr, *lam = nullptr, *W = nullptr;
  const int* map1d = nullptr;
  T inv_wend = 0;
};
struct BatchLaunch {
  int nb = 0;           // buckets
  int ntiles = 0;       // tiles of the stage
  int grid = 0;         // workgroups (a multiple of 8)
  bool persistent = false;   // fewer workgroups than tiles: each strides through the list
};
enum { kStageOp = 0, kStageSolve = 1, kStageAdd = 2 };
// tiles per bucket of each stage (elements per tile times right-hand sides)
int stage_tiles(int stage, int p, int nel, int nrhs);
// workgroup size of the batched kernel of a stage for largest degree pmax
int stage_threads(int stage, int pmax);
template <typename T>
void sipg_apply_batched(int pmax, const OpArgs<T>& a, const BucketDesc<T>* bd, const BatchLaunch& l, hipStream_t st);

// one-time geometry of a degree bucket (Sec. 2.2)
struct GeoArgs {
  int nel = 0;
  const int* elist = nullptr;       // [nel] element ids (null: 0..nel-1)
  const int64_t* off = nullptr;     // [E] first node per element (null: e (p+1)^3)
  const int64_t* offF = nullptr;    // [E] first face-node slot per element (null: 6 e (p+1)^2)
  int64_t ndof = 0;                 // nodes of the level (stride of G)
  const double* X = nullptr;        // coordinates, element e at 3 off[e]: [3][(p+1)^3]
  double *G = nullptr, *WJ = nullptr, *ws = nullptr, *vol = nullptr, *area = nullptr, *lin = nullptr;
  int* bad = nullptr;               // set when det J <= 0 somewhere
  const double* nun = nullptr;      // nodal diffusivity (null: the scalar nu everywhere)
  double* nuavg = nullptr;          // [E] element average of nu (int nu dx / int dx), or null
};
void geometry(int p, const GeoArgs& g, const double* D, const double* w, const double* x, double nu,
              hipStream_t st);

struct RhsArgs {
  int nel = 0;
  const int* elist = nullptr;
  const int64_t* off = nullptr;
  const int64_t* offF = nullptr;
  int64_t ndof = 0;
  const double *f = nullptr, *uD = nullptr, *qN = nullptr;
  double* b = nullptr;
  const double *G = nullptr, *WJ = nullptr, *pen = nullptr, *ws = nullptr;
  const int* nbr = nullptr;
  const int8_t* bc = nullptr;
};
void rhs(int p, const RhsArgs& r, const double* D, double inv_wend, hipStream_t st);

// nun: nodal diffusivity (uniform degree, offsets e (p+1)^3) or null for the scalar nu
void penalty(int E, int p, const int* deg, const int64_t* offF, double mu_star, double nu, const double* nun,
             const int* nbr, const int8_t* nfo,
             const int8_t* bc, const double* vol, const double* area, const double* ws, double* pen, double* muf,
             hipStream_t st);

// Face terms of the faces between elements of different degree (mixed-degree levels):
// integrated on the finer side's face grid, added to (mode 1) or subtracted from (mode 0)
// the output of sipg_apply, which leaves these faces out.
template <typename T>
struct MortarArgs {
  int nrhs = 1;
  int64_t ndof = 0;
  const T* u = nullptr;
  const T* G = nullptr;             // [6][ndof]
  const double* ws = nullptr;       // face omega s, [offF]
  const double* muf = nullptr;      // [E][6] mu_F nu
  const double* Dall = nullptr;     // differentiation matrices of degrees 1..8, degree p at (p-1) * 81
  const double* Iall = nullptr;     // interpolation degree q -> r at ((q-1) * 8 + (r-1)) * 81
  int nface = 0;                    // faces between degrees (one task per face, both sides)
  // [nface][8] per face: e * 6 + phi of its lower-id side e, the neighbour en, the degrees of e
  // and en, then the first DOF and the first face-node slot of e and of en
  const int64_t* fdesc = nullptr;
  void* fres = nullptr;             // [nrhs][2 nface][kMortarFaceRes] T: row and lifting terms per side
};
// The face terms of every face between degrees, into fres; the operator kernels of the level
// then add them (OpArgs::fmapE / fres), so this runs before them.
template <typename T>
void sipg_mortar_faces(const MortarArgs<T>& a, hipStream_t st);

// Schwarz method on unstructured meshes (Sec. 4.3.1 with oriented faces and irregular edges and
// vertices): the subdomain tiles are gathered through per-slot tables built on the host, and the
// corrections are summed per node from the stored tiles.
template <typename T>
struct TopoArgs {
  int nel = 0;                    // subdomains (the elements of the level)
  int nrhs = 1;                   // vectors are [nrhs][ndof], tiles [nrhs][nel][nt]
  int nt = 0;                     // slots per tile, ns^3
  int64_t ndof = 0;
  const T* r = nullptr;
  T* z = nullptr;
  int mode = 0;                   // 0: z = B r, 1: z += B r
  const int* gather = nullptr;    // [nel][nt] node of each slot, -1 zero, -2 - j merged slot j
  const int* mptr = nullptr;      // [merged slots + 1] into midx
  const int* midx = nullptr;      // the nodes averaged into each merged slot
  const int8_t* var = nullptr;    // [nel][3] 1D variant per direction
  const T* S = nullptr;           // [variants][ns][ns] eigenvectors S[c][q], zero-padded
  const T* ST = nullptr;          // their transposes
  const T* lam = nullptr;         // [variants][ns] eigenvalues
  const T* gco = nullptr;         // [nel][4] surrogate coefficients g0..g3
  T* Zt = nullptr;                // [nrhs][nel][nt] subdomain solutions
  const int64_t* sptr = nullptr;  // [ndof + 1] per node into sslot / scoef
  const int* sslot = nullptr;     // subdomain * nt + slot of every contribution to the node
  const T* scoef = nullptr;       // its weight: merge share x tensor weight x 1 / weight sum
};

template <typename T>
void topo_schwarz_solve(int ns, const TopoArgs<T>& a, hipStream_t st);
template <typename T>
void topo_schwarz_scatter(const TopoArgs<T>& a, hipStream_t st);

template <typename T>
struct SchwarzArgs {
  int E = 0;
  int nrhs = 1;               // vectors are [nrhs][ndof], inbox [nrhs][nin]
  int nel = 0;                // subdomains of this launch (the degree bucket)
  const int* elist = nullptr; // [nel] element ids (null: 0..nel-1)
  const int64_t* off = nullptr;   // [E] first DOF per element (null: uniform)
  const int64_t* offO = nullptr;  // [E] first inbox slot per element (null: uniform)
  const int* deg = nullptr;   // [E] degree per element (null: uniform)
  int64_t ndof = 0;           // DOF per right-hand side
  int64_t nin = 0;            // inbox slots per right-hand side
  const T* r = nullptr;       // input residual
  T* z = nullptr;             // output (mode 0: z = own part; mode 1: z += own part)
  int mode = 0;
  T* O = nullptr;             // overlap buffer [E][osz]
  const int* nb27 = nullptr;  // [E][27]
  const int8_t* var = nullptr;   // [E][3] variant index (left * 4 + right, sides I, D, N, I0)
  const T* gco = nullptr;     // [E][4] g0..g3
  const T* S = nullptr;       // [16][ns*ns] padded eigenvector tables, S[i*ns + a] = (s_a)_i
  const T* ST = nullptr;      // [16][ns*ns] transposes
  const T* lam = nullptr;     // [16][ns]
  const T* W = nullptr;       // [16][ns]
  const int* map1d = nullptr; // [16][ns]: (delta+1)*64 + loc, or -1 for padding
  const T* cinv = nullptr;    // [ndof] 1 / (sum of the subdomain weights at the node) on levels
                              // whose tensor weights do not add up to one (degree jumps); null: 1
  const uint8_t* sel = nullptr;  // [E] subdomains to solve (null: all)
  int unweighted = 0;            // 1: W = I (block-diagonal local solves)
  const float* corr = nullptr;   // [E][ns^3] learned correction added to the FD tile (or null)
  const double* cscale = nullptr;  // [E] scale of corr (the subdomain residual norm)
  // overlap add only: z^T dr and z^T (dr - dr0) of the final z summed per tile into
  // dotz / dotz2 [nrhs][tiles] (dotz null: no dot products; dr0 null: z^T dr only)
  const T* dr = nullptr;
  const T* dr0 = nullptr;
  double* dotz = nullptr;
  double* dotz2 = nullptr;
};

// Learned-correction helpers over the subdomain tiles of a list of elements (null list: all)
template <typename T>
void tile_features(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, const double* v, const double* J9,
                   float* X, double* norms, hipStream_t st);
template <typename T>
void tile_diff(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, const double* v1, const double* v2,
               const double* norms, float* out, hipStream_t st);
template <typename T>
void mark_subdomains(int p, int m, const SchwarzArgs<T>& a, const int* ids, int n, double* mask, hipStream_t st);

template <typename T>
void schwarz_solve(int p, int m, const SchwarzArgs<T>& a, hipStream_t st);
template <typename T>
void schwarz_overlap_add(int p, int m, const SchwarzArgs<T>& a, hipStream_t st);
int overlap_size(int p, int m);
// FP32 subdomain solve with the contractions on BF16 (bf16) or FP32 matrix cores (overlap 1);
// false when the arguments ask for something it does not do (masked, weighted-off or learned)
bool schwarz_solve_mfma(int p, int m, const SchwarzArgs<float>& a, bool bf16, hipStream_t st);
template <typename T>
void schwarz_solve_batched(int pmax, const SchwarzArgs<T>& a, const BucketDesc<T>* bd, const BatchLaunch& l,
                           hipStream_t st);
template <typename T>
void schwarz_overlap_add_batched(int pmax, const SchwarzArgs<T>& a, const BucketDesc<T>* bd, const BatchLaunch& l,
                                 hipStream_t st);

// transfers: out (=|+=) T(x)T(x)T (in - in2) per element; T is n_out x n_in
template <typename T>
struct XferArgs {
  int nel = 0;                       // elements of this launch
  const int* elist = nullptr;        // [nel] element ids (null: 0..nel-1)
  const int64_t* off_in = nullptr;   // [E] first input node per element (null: e n_in^3)
  const int64_t* off_out = nullptr;  // [E] first output node per element (null: e n_out^3)
  int ncomp = 1;                     // components stored per element (3 for coordinates)
  int nrhs = 1;
  int64_t stride_in = 0, stride_out = 0;  // right-hand-side strides
  const T* Tm = nullptr;
  const T* in = nullptr;
  const T* in2 = nullptr;            // subtracted from in when non-null
  T* out = nullptr;
  int accumulate = 0;
};
template <typename T>
bool tensor3(int n_in, int n_out, const XferArgs<T>& a, hipStream_t st);

// Transfers across one h-coarsening (Sec. 3.2) on uniform levels of degree N - 1: a parent and
// its eight children c = bx + 2 by + 4 bz, child b covering xi in [-1, 0] (b = 0) or [0, 1] of
// the parent in each direction.  kind 0: out = P in (children -> parent, the children's fields at
// the parent's nodes, averaged where shared); 1: out (=|+=) R in, R = I^T; 2: out (=|+=) I (in - in2)
// (parent -> children).  Element e's block of component c and right-hand side k starts at
// k stride + (e ncomp + c) N^3.
template <typename T>
struct HXferArgs {
  int kind = 0;
  int ncoarse = 0;                   // parents of this launch
  const int* parents = nullptr;      // [ncoarse] parent element ids (null: 0..ncoarse-1)
  const int* children = nullptr;     // [ncoarse][8] fine element ids, row i for parents[i]
  int ncomp = 1, nrhs = 1;
  int64_t stride_f = 0, stride_c = 0;
  const T* M = nullptr;              // [6][N][N]: P_0, P_1, R_0 = I_0^T, R_1 = I_1^T, I_0, I_1
  const T* in = nullptr;
  const T* in2 = nullptr;            // subtracted from in when non-null (kind 2)
  T* out = nullptr;
  int accumulate = 0;                // add to out
};
// dst rows of the listed elements = src rows (n3 values per element, uniform layout)
void copy_rows(const int* list, int n, int n3, const double* src, double* dst, hipStream_t st);
// out[i] = sum of squares of v over element list[i] (n3 values per element, uniform layout)
void rows_sumsq(const int* list, int n, int n3, const double* v, double* out, hipStream_t st);
template <typename T>
bool htransfer(int p, const HXferArgs<T>& a, hipStream_t st);

int reduction_blocks(int64_t n);

}  // namespace dgfas
