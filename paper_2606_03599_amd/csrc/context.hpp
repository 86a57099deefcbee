// Context of libpbr: grid, material on the device (natural layout and the four
// parity-block layouts), per-layout work buffers and the kernel entry points
// used by the solver drivers.
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include "../../include/pbr.h"
#include "common.hpp"
#include "geometry.hpp"

// k-points whose solves can run in lockstep (each with its own work areas and
// FFT tables), and layouts batched into one launch at most: 4 blocks per k-point.
#define PBR_KSLOTS 4
#define PBR_MAX_BATCH (4 * PBR_KSLOTS)
// Doubles of pinned host scratch per context.
#define PBR_PINNED 32768
#define PBR_TUNE_SLOTS 16

// Device material in one layout: C as 21 planes of N doubles (SoA), rho, sqrt(rho).
// Stiffness as the stencil reads it: for every row (j, k) of the layout box and
// every run of PBR_CT_W consecutive i, the 21 stiffness entries and rho of
// those nodes, entry-major (22 x PBR_CT_W doubles, 2816 bytes, contiguous):
//   Ct[(((k * L2 + j) * tiles + i / PBR_CT_W) * 22 + q) * PBR_CT_W + i % PBR_CT_W]
// with tiles = ceil(L1 / PBR_CT_W), q < 21 the C21 entry, q = 21 rho; nodes past
// L1 in the last run hold zeros.  One wave's loads of one entry for a 16 x 4
// patch of nodes are then four 128-byte segments, and a row's 22 entries are
// one contiguous 2.8 KB run of HBM.
#define PBR_CT_W 16
// Palette form of the same data: when the material has at most PBR_PAL_MAX
// distinct (C21, rho) rows, every layout also holds one byte per node (its row
// in the palette, layout order) and the context holds the palette, 22 doubles
// per row in the order of Ct's entries.  The stencil then reads one byte per
// node instead of 176 and takes the row from LDS; the values, and therefore
// every operator output, are the same bit for bit.
#define PBR_PAL_MAX 256

struct DevMaterial {
  long N = 0;
  long ct_len = 0;          // doubles in Ct
  double* Ct = nullptr;     // stencil tiles (layout above)
  unsigned char* idx = nullptr;  // [N] palette row of each node (valid when npal > 0)
  double* rho = nullptr;    // [N]
  double* srho = nullptr;   // [N]  sqrt(rho)
  double* isrho = nullptr;  // [N]  1/sqrt(rho)
};

// Per-kappa tables of the FFT preconditioner for one layout.
struct FftTables {
  double kappa[3] = {1e300, 1e300, 1e300};
  cplx* twist[3] = {nullptr, nullptr, nullptr};   // e^{-i x phi_l / L_l}, x in [0,L_l)
  cplx* post[3] = {nullptr, nullptr, nullptr};    // e^{-i beta_q} per frequency (block y2/y3)
  cplx* roots[3] = {nullptr, nullptr, nullptr};   // e^{-2 pi i k / L_l}
  // blocks with the three-pass preconditioner: e^{i alpha}, e^{i beta},
  // e^{i gamma} in the digit-reversed order its transforms leave along i', y2
  // and y3 (lengths n1/2, n2/2, n3/2)
  cplx* postp[3] = {nullptr, nullptr, nullptr};
  int L[3] = {0, 0, 0};
};

struct PcgScalars;

// Work buffers of one layout (allocated on first use).
struct LayoutWork {
  long N = 0;                 // nodes
  cplx *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
  cplx *b = nullptr, *w = nullptr, *t = nullptr;   // Lanczos / staging vectors
  cplx *U = nullptr, *U2 = nullptr;                // Krylov bases (3N x ucols)
  int ucols = 0;
  int ritz_n = 0;  // Ritz vectors (M^1/2-scaled) of the last finished run held in U2
  cplx* small = nullptr;      // small device matrices (h, Y), 4096 complex
  double* part = nullptr;     // reduction partials
  double* part2 = nullptr;
  double* dscal = nullptr;    // small device scalars (256 doubles)
  PcgScalars* st = nullptr;
  double* ppart = nullptr;    // fused PCG partials: 3 buffers of pcap doubles
  long pcap = 0;
  double* Wnull = nullptr;    // Gamma null fields (nf x N real, orthonormal after sqrt(rho))
  int nf = 0;
  int block = -2;             // layout of this work area (-1 full, 0..3 blocks)
};

struct pbr_ctx {
  int n1 = 0, n2 = 0, n3 = 0;
  long n = 0;
  bool even = false;
  double Alat[9];      // column-major
  double Ainv[9];      // row-major: Ainv[s*3+m] = (A_lat^-1)_{sm}
  double cf[3][5];     // Cartesian stencil coefficients
  int device = 0;
  int cus = 256;       // compute units of the device
  // stencil chunk lengths chosen by the autotuner, per (batch size, box)
  struct StencilTune {
    int nb = 0, L1 = 0, L2 = 0, L3 = 0, pal = 0, pin_ti = 0, pin_tj = 0;
    int ti = 0, tj = 0, chunk = 0;
  } stencil_tune[PBR_TUNE_SLOTS];
  int stencil_tune_next = 0;
  // i-width of the block mode-solve pass chosen per (batch size, box)
  struct SolveTune {
    int nb = 0, L1 = 0, L2 = 0, L3 = 0, bi = 0;
  } solve_tune[PBR_TUNE_SLOTS];
  int solve_tune_next = 0;
  int pin_ti = 0, pin_tj = 0;  // stencil tile shape pinned by pbr_set_stencil_shape (0: tuned)
  int precond_passes = 0;      // pbr_set_precond_passes: 0 automatic, 3 or 5
  int pin_bi = 0;              // mode-solve i-width pinned by pbr_set_solve_width (0: tuned)
  hipStream_t stream = nullptr;
  bool own_stream = false;

  bool have_material = false;
  double Cmax = 0.0;
  double Cref[21];
  double rho_ref = 1.0;
  std::vector<double> rho_host;   // natural order
  DevMaterial mat[5];  // index 0 = natural (full), 1..4 = blocks 0..3
  int npal = 0;              // palette rows (0: the material has more than PBR_PAL_MAX)
  double* pal = nullptr;     // PBR_PAL_MAX x 22 doubles on the device
  bool use_palette = true;   // pbr_set_palette
  int pcg_hint = 0;          // PCG iterations of the last fused solve (first host check)
  // Bumped whenever the material, the reference material or the stiffness
  // form changes: launch arguments captured in a graph depend on all three.
  unsigned long mat_gen = 0;
  FftTables fft[2 * PBR_KSLOTS];     // [slot][natural, blocks]
  LayoutWork work[5 * PBR_KSLOTS];   // [slot][natural, block 0..3]

  double* hpinned = nullptr;      // pinned host scratch (PBR_PINNED doubles)
  cplx* scratch = nullptr;        // this device's fixed table array (pbr_precond_noalloc)
  PcgScalars* st_all = nullptr;   // device CG scalars of all work areas, contiguous
  // One captured chunk of fused PCG iterations, replayed while its launch
  // arguments (layouts, vectors, k, shift, chunk length) stay the same.
  struct PcgGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int nb = 0, chunk = 0;
    int blocks[PBR_MAX_BATCH] = {};
    int slots[PBR_MAX_BATCH] = {};
    double kap[PBR_MAX_BATCH][3] = {};
    const void* b[PBR_MAX_BATCH] = {};
    const void* x[PBR_MAX_BATCH] = {};
    double shift = 0.0;
    unsigned long mat_gen = 0;
  } pcg_graph;
  hipStream_t cap_stream = nullptr;  // capture stream (the context stream may be the null stream)
  bool graphs_broken = false;        // capture failed once: launch eagerly from then on

  std::string err;
  std::mutex err_mu;
  void set_error(const std::string& s) {
    std::lock_guard<std::mutex> lk(err_mu);
    err = s;
  }

  DevMaterial& material(int block) { return mat[block + 1]; }
  LayoutWork& wk(int slot, int block) { return work[5 * slot + block + 1]; }
  FftTables& tables(int slot, bool blocked) { return fft[2 * slot + (blocked ? 1 : 0)]; }
  long layout_nodes(int block) const { return block < 0 ? n : n / 4; }
};

// ---- kernels / device helpers (implemented in the .hip files) ----
int dev_alloc(pbr_ctx* c, void** p, size_t bytes);
void dev_free(void* p);
int upload_material(pbr_ctx* c, const double* C21_host, const double* rho_host);
int layout_gather(pbr_ctx* c, int block, const cplx* full, cplx* blk);
int layout_scatter(pbr_ctx* c, int block, const cplx* blk, cplx* full);

// Geometry of a layout at wave vector kappa.
Geo make_geo(const pbr_ctx* c, int block, const double kappa[3]);
// One fused PCG iteration's preconditioner work (see PcgHook): x, r updated
// with alpha from the (p, q) partials of the matvec (or r = b, x = 0 at init),
// z the transform buffer, pout = z + beta p (p at init).
struct PcgStep {
  int slot = 0;       // work area / FFT tables of this layout's k-point
  int block = -1;
  double kappa[3] = {0, 0, 0};
  PcgScalars* st = nullptr;
  int init = 0;
  double tol2 = 0.0;
  cplx* x = nullptr;
  cplx* r = nullptr;
  const cplx* p = nullptr;
  const cplx* q = nullptr;
  const cplx* b = nullptr;
  cplx* z = nullptr;
  cplx* pout = nullptr;
  const double* part_pq = nullptr;
  int n_pq = 0;
  double* part_rr = nullptr;
  double* part_rz = nullptr;
  long part_cap = 0;  // capacity of each partial buffer (doubles)
};

// One layout of a batched matvec: y = (A + s M) x in layout `block`.  With st
// non-null its work-groups do nothing once st->done != 0 and write partials of
// Re(x^H y) to part.
struct ApplyLayout {
  int block = -1;
  cplx ph[3] = {{1, 0}, {1, 0}, {1, 0}};  // e^{i phi_l} of this layout's k
  const cplx* x = nullptr;
  cplx* y = nullptr;
  PcgScalars* st = nullptr;
  double* part = nullptr;
};
// nb layouts of one kind (parity blocks, or natural layouts) in one launch;
// g is the geometry of any of them (class bits and Bloch phases come from L[t]);
// *nparts receives the partials per layout.
// whether the stencil's work split for this batch size and box is tuned already
bool apply_tuned(const pbr_ctx* c, const Geo& g, int nb);
// (x, y) partials one matvec launch writes per layout (block -1: natural)
long apply_partials(const pbr_ctx* c, int block);
int launch_apply_batch(pbr_ctx* c, const Geo& g, int nb, const ApplyLayout* L, double s,
                       long part_cap = 0, int* nparts = nullptr);
int launch_apply(pbr_ctx* c, const Geo& g, int block, double s, const cplx* x, cplx* y,
                 PcgScalars* st = nullptr, double* part = nullptr, long part_cap = 0,
                 int* nparts = nullptr);
// z = preconditioner(r) in layout `block`
int launch_precond(pbr_ctx* c, const double kappa[3], int block, double shift,
                   const cplx* r, cplx* z);
// The same with the tables in the device's fixed scratch array (no allocation;
// n_l <= 256), and the one-time lookup of that array's address per device.
int launch_precond_noalloc(pbr_ctx* c, const double kappa[3], int block, double shift,
                           const cplx* r, cplx* z);
int scratch_init(pbr_ctx* c);
// The preconditioner passes of one fused PCG iteration (five launches) for nb
// layouts of one kind at once; P[t] names the layout (slot, block, kappa).
int launch_pcg_precond_batch(pbr_ctx* c, int nb, const PcgStep* P, double shift);

// A layout of a batched solve: work area (slot, block) at wave vector kappa.
struct LayoutRef {
  int slot = 0;
  int block = -1;
  double kappa[3] = {0, 0, 0};
  int warm_slot = -1;  // start from the Ritz vectors held by work area (warm_slot, block)
};

// Adds sum_s w[s] d lambda_s / d (C21, rho) of nvec M-normalised eigenvectors v
// (vector-major, layout `block`) to the natural-order fields gC (n x 21), grho.
int launch_eig_grad(pbr_ctx* c, const Geo& g, int block, int nvec, const double* lam,
                    const double* w, const cplx* v, double* gC, double* grho);

// streaming copy of `bytes` (a multiple of 16) on the context stream (probe.hip)
int launch_copy_probe(pbr_ctx* c, const void* src, void* dst, long bytes);

// One kernel of each source file queried on the calling thread, so that the
// runtime loads every code object of the library onto the device there (at
// pbr_create) rather than at a first launch, which several host threads may
// issue at once (pbr_band_paths).
int preload_stencil(pbr_ctx* c);
int preload_fft(pbr_ctx* c);
int preload_blas(pbr_ctx* c);
int preload_layout(pbr_ctx* c);
int preload_grad(pbr_ctx* c);
int preload_probe(pbr_ctx* c);
inline int preload_kernels(pbr_ctx* c) {
  PBR_TRY(preload_stencil(c));
  PBR_TRY(preload_fft(c));
  PBR_TRY(preload_blas(c));
  PBR_TRY(preload_layout(c));
  PBR_TRY(preload_grad(c));
  return preload_probe(c);
}

// solver drivers (solver.cpp)
int ensure_work(pbr_ctx* c, int slot, int block);
int pcg_solve(pbr_ctx* c, int block, const double kappa[3], double shift, const cplx* b, cplx* x,
              const pbr_opts& o, int* iters, int* conv);
int lanczos_eigs(pbr_ctx* c, const double kappa[3], int block, int nev, double shift,
                 const pbr_opts& o, double* evals, cplx* evecs_dev, pbr_stats* st);
// evecs_dev (optional, with blocks_out): the merged eigenpairs' block-layout
// eigenvectors, nev x 3n/4 complex vector-major, and the block of each.
int merged_eigs(pbr_ctx* c, const double kappa[3], int nev, double shift, const pbr_opts& o,
                double* evals, pbr_stats* st, cplx* evecs_dev = nullptr,
                int* blocks_out = nullptr);
// Blocked (certified merge) and full-space eigenvalues along nk wave vectors
// (kappas: nk x 3, evals: nk x nev), up to PBR_KSLOTS k-points in lockstep.
int merged_path(pbr_ctx* c, int nk, const double* kappas, int nev, double shift,
                const pbr_opts& o, double* evals, pbr_stats* st, cplx* evecs_dev = nullptr,
                int* blocks_out = nullptr);
int full_path(pbr_ctx* c, int nk, const double* kappas, int nev, double shift,
              const pbr_opts& o, double* evals, pbr_stats* st);
