// Solver drivers: the inner preconditioned CG for (A + shift M) x = b
// (Sec. 6.1, Eq. 6.2) and the outer thick-restart Lanczos (Krylov-Schur for a
// Hermitian operator) on the shift-invert operator (Sec. 6.1), with the Gamma
// zero-derivative modes projected out (Sec. 6.2, Appendix C), the block merge
// with certification, and the Bloch path loop.
//
// The outer iteration works in the M^{1/2}-scaled space: with u = M^{1/2} v the
// pencil (A, M) becomes the Hermitian operator Op = M^{1/2} (A + shift M)^{-1}
// M^{1/2} with eigenvalues mu = 1/(lambda + shift) and Euclidean-orthonormal
// Krylov bases.  One application of Op is one PCG solve.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "../../include/pbr_host.h"
#include "blas.hpp"
#include "context.hpp"

typedef std::complex<double> zc;

namespace {

constexpr int SMALL_CPLX = 8192;  // capacity of LayoutWork::small
constexpr int NSTATE = 5 * PBR_KSLOTS;  // device CG scalar sets (one per work area)

int alloc_vec(pbr_ctx* c, cplx** p, long n3) { return dev_alloc(c, (void**)p, sizeof(cplx) * n3); }

// Grows the Krylov bases to cols columns.  The Ritz vectors a finished run left
// in U2 move to the new U2: a later run's warm start reads them (a block solved
// again with more eigenpairs needs a larger basis and starts from its own
// earlier Ritz vectors), and dropping them would make that start depend on
// whether an earlier call had already grown the basis.
int ensure_basis(pbr_ctx* c, LayoutWork& W, int cols) {
  if (W.ucols >= cols) return ST_OK;
  cplx* old2 = W.U2;
  const int keep = old2 ? std::min(W.ritz_n, W.ucols) : 0;
  dev_free(W.U);
  W.U = W.U2 = nullptr;
  W.ucols = 0;
  W.ritz_n = 0;
  const long n3 = 3 * W.N;
  int rc = alloc_vec(c, &W.U, n3 * (long)cols);
  if (rc == ST_OK) rc = alloc_vec(c, &W.U2, n3 * (long)cols);
  if (rc == ST_OK && keep > 0) {
    hipError_t e = hipMemcpyAsync(W.U2, old2, sizeof(cplx) * n3 * keep, hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      c->set_error(std::string("Ritz vector copy: ") + hipGetErrorString(e));
      rc = ST_EDEVICE;
    } else {
      W.ritz_n = keep;
    }
  }
  dev_free(old2);
  if (rc != ST_OK) {
    dev_free(W.U);
    dev_free(W.U2);
    W.U = W.U2 = nullptr;
    W.ritz_n = 0;
    return rc;
  }
  W.ucols = cols;
  return ST_OK;
}

bool is_gamma(const double k[3]) {
  for (int l = 0; l < 3; ++l)
    if (k[l] != std::round(k[l])) return false;
  return true;
}

// Read `count` doubles from device to host (synchronises the stream).
int readback(pbr_ctx* c, const double* dev, double* host, int count) {
  if (count > PBR_PINNED) {
    c->set_error("readback larger than the pinned staging buffer");
    return ST_EINVAL;
  }
  PBR_HIP(c, hipMemcpyAsync(c->hpinned, dev, sizeof(double) * count, hipMemcpyDeviceToHost,
                            c->stream));
  PBR_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < count; ++i) host[i] = c->hpinned[i];
  return ST_OK;
}

int upload_small(pbr_ctx* c, cplx* dev, const std::vector<zc>& h) {
  if ((long)h.size() > SMALL_CPLX || 2 * (long)h.size() > PBR_PINNED) {
    c->set_error("Krylov basis too large for the small-matrix buffer");
    return ST_EINVAL;
  }
  for (size_t i = 0; i < h.size(); ++i) {
    c->hpinned[2 * i] = h[i].real();
    c->hpinned[2 * i + 1] = h[i].imag();
  }
  PBR_HIP(c, hipMemcpyAsync(dev, c->hpinned, sizeof(cplx) * h.size(), hipMemcpyHostToDevice,
                            c->stream));
  // the pinned staging buffer is reused by the next call: wait for the copy
  PBR_HIP(c, hipStreamSynchronize(c->stream));
  return ST_OK;
}

// Gamma null fields of a layout: nf real fields w_f with sum_t w_f w_g = delta_fg
// such that {sqrt(rho) chi e_alpha} = span{w_f e_alpha}: the M^{1/2} image of an
// M-orthonormal basis of N_Gamma.  Full space: chi in {1, (-1)^{i+j},
// (-1)^{i+k}, (-1)^{j+k}} (4 fields); a block: all four are +-1 on the class,
// so one field sqrt(rho)/sqrt(sum rho).
int ensure_null_fields(pbr_ctx* c, int slot, int block) {
  LayoutWork& W = c->wk(slot, block);
  if (W.Wnull) return ST_OK;
  const long N = W.N;
  std::vector<double> rho(N);
  const int n1 = c->n1, n2 = c->n2, m2 = c->n2 / 2;
  if (block < 0) {
    rho = c->rho_host;
  } else {
    const int a = block >> 1, cc = block & 1;
    for (long t = 0; t < N; ++t) {
      const int i = (int)(t % n1);
      const long r = t / n1;
      const int y2 = (int)(r % m2), y3 = (int)(r / m2);
      const int j = 2 * y2 + ((a + i) & 1), k = 2 * y3 + ((a + cc + i) & 1);
      rho[t] = c->rho_host[(size_t)i + (size_t)n1 * ((size_t)j + (size_t)n2 * k)];
    }
  }
  std::vector<double> F;
  int nf;
  if (block < 0) {
    nf = 4;
    F.assign((size_t)4 * N, 0.0);
    std::vector<double> chi((size_t)4 * N);
    for (long t = 0; t < N; ++t) {
      const int i = (int)(t % n1);
      const long r = t / n1;
      const int j = (int)(r % n2), k = (int)(r / n2);
      chi[t] = 1.0;
      chi[N + t] = ((i + j) & 1) ? -1.0 : 1.0;
      chi[2 * N + t] = ((i + k) & 1) ? -1.0 : 1.0;
      chi[3 * N + t] = ((j + k) & 1) ? -1.0 : 1.0;
    }
    // Gram G = chi^T diag(rho) chi, Cholesky G = L L^T, fields = sqrt(rho) chi L^{-T}
    double G[4][4] = {};
    for (int f = 0; f < 4; ++f)
      for (int g = 0; g < 4; ++g) {
        double s = 0.0;
        for (long t = 0; t < N; ++t) s += rho[t] * chi[f * N + t] * chi[g * N + t];
        G[f][g] = s;
      }
    double L[4][4] = {};
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = G[i][j];
        for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
        if (i == j) {
          if (s <= 0) {
            c->set_error("Gamma null space Gram matrix not positive (grid too small?)");
            return ST_EINVAL;
          }
          L[i][i] = std::sqrt(s);
        } else {
          L[i][j] = s / L[j][j];
        }
      }
    // Linv (lower)
    double Li[4][4] = {};
    for (int i = 0; i < 4; ++i) {
      Li[i][i] = 1.0 / L[i][i];
      for (int j = 0; j < i; ++j) {
        double s = 0.0;
        for (int k = j; k < i; ++k) s += L[i][k] * Li[k][j];
        Li[i][j] = -s / L[i][i];
      }
    }
    // field g = sqrt(rho) * sum_f chi_f (L^{-T})[f][g] = sqrt(rho) sum_f chi_f Li[g][f]
    for (int g = 0; g < 4; ++g)
      for (long t = 0; t < N; ++t) {
        double s = 0.0;
        for (int f = 0; f < 4; ++f) s += chi[f * N + t] * Li[g][f];
        F[(size_t)g * N + t] = std::sqrt(rho[t]) * s;
      }
  } else {
    nf = 1;
    F.assign(N, 0.0);
    double sr = 0.0;
    for (long t = 0; t < N; ++t) sr += rho[t];
    for (long t = 0; t < N; ++t) F[t] = std::sqrt(rho[t] / sr);
  }
  PBR_TRY(dev_alloc(c, (void**)&W.Wnull, sizeof(double) * nf * N));
  PBR_HIP(c, hipMemcpyAsync(W.Wnull, F.data(), sizeof(double) * nf * N, hipMemcpyHostToDevice,
                            c->stream));
  PBR_HIP(c, hipStreamSynchronize(c->stream));
  W.nf = nf;
  return ST_OK;
}

int project_null(pbr_ctx* c, LayoutWork& W, cplx* v) {
  return proj_gamma(c, c->stream, W.N, W.nf, W.Wnull, v, W.part, W.dscal);
}

double vnorm(pbr_ctx* c, LayoutWork& W, const cplx* v, int* status) {
  double h;
  int s = dot_real_async(c, c->stream, 3 * W.N, v, v, W.part, W.dscal);
  if (s == ST_OK) s = readback(c, W.dscal, &h, 1);
  *status = s;
  return std::sqrt(std::max(h, 0.0));
}

}  // namespace

int ensure_work(pbr_ctx* c, int slot, int block) {
  LayoutWork& W = c->wk(slot, block);
  const long N = c->layout_nodes(block);
  if (W.N == N && W.x) return ST_OK;
  W.N = N;
  W.block = block;
  const long n3 = 3 * N;
  PBR_TRY(alloc_vec(c, &W.x, n3));
  PBR_TRY(alloc_vec(c, &W.r, n3));
  PBR_TRY(alloc_vec(c, &W.p, n3));
  PBR_TRY(alloc_vec(c, &W.q, n3));
  PBR_TRY(alloc_vec(c, &W.z, n3));
  PBR_TRY(alloc_vec(c, &W.b, n3));
  PBR_TRY(alloc_vec(c, &W.w, n3));
  PBR_TRY(alloc_vec(c, &W.t, n3));
  PBR_TRY(dev_alloc(c, (void**)&W.small, sizeof(cplx) * SMALL_CPLX));
  PBR_TRY(dev_alloc(c, (void**)&W.part, sizeof(double) * 1024 * 2 * 128));
  PBR_TRY(dev_alloc(c, (void**)&W.part2, sizeof(double) * 1024 * 2));
  PBR_TRY(dev_alloc(c, (void**)&W.dscal, sizeof(double) * 4096));
  if (!c->st_all) PBR_TRY(dev_alloc(c, (void**)&c->st_all, sizeof(PcgScalars) * NSTATE));
  W.st = c->st_all + (5 * slot + block + 1);
  W.pcap = N / 128 + 4096 + apply_partials(c, block);
  PBR_TRY(dev_alloc(c, (void**)&W.ppart, sizeof(double) * 3 * W.pcap));
  return ST_OK;
}

namespace {

// Device CG scalars of all work areas in one copy.
int read_states(pbr_ctx* c, PcgScalars hs[NSTATE]) {
  static_assert(sizeof(PcgScalars) * NSTATE <= sizeof(double) * PBR_PINNED, "staging");
  PBR_HIP(c, hipMemcpyAsync(c->hpinned, c->st_all, sizeof(PcgScalars) * NSTATE,
                            hipMemcpyDeviceToHost, c->stream));
  PBR_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(hs, c->hpinned, sizeof(PcgScalars) * NSTATE);
  return ST_OK;
}

int state_index(int slot, int block) { return 5 * slot + block + 1; }

// Unpreconditioned CG of one layout (kept for pbr_opts.precond = 0).
int pcg_plain(pbr_ctx* c, int slot, int block, const double kappa[3], double shift,
              const cplx* b, cplx* x, const pbr_opts& o) {
  LayoutWork& W = c->wk(slot, block);
  const hipStream_t SO = c->stream;
  const long n3 = 3 * W.N;
  const Geo g = make_geo(c, block, kappa);
  const int chunk = o.check_every > 0 ? o.check_every : 10;
  PBR_TRY(vec_zero(c, SO, n3, x));
  PBR_TRY(vec_copy(c, SO, n3, b, W.r));
  PBR_TRY(vec_copy(c, SO, n3, W.r, W.z));
  PBR_TRY(vec_copy(c, SO, n3, W.z, W.p));
  PBR_TRY(pcg_init_async(c, SO, n3, W.r, W.z, o.tol_inner, W.part, W.part2, W.st));
  int done_iters = 0;
  PcgScalars hs[NSTATE];
  const int si = state_index(slot, block);
  for (;;) {
    const int todo = std::min(chunk, o.maxit_inner - done_iters);
    if (todo <= 0) break;
    for (int it = 0; it < todo; ++it) {
      PBR_TRY(launch_apply(c, g, block, shift, W.p, W.q, W.st));
      PBR_TRY(pcg_alpha(c, SO, n3, W.p, W.q, W.part, W.st));
      PBR_TRY(pcg_xr(c, SO, n3, x, W.r, W.p, W.q, W.part, W.st));
      PBR_TRY(vec_copy(c, SO, n3, W.r, W.z));
      PBR_TRY(pcg_beta_p(c, SO, n3, W.r, W.z, W.p, W.part, W.st));
    }
    PBR_TRY(read_states(c, hs));
    done_iters = hs[si].iters;
    if (hs[si].done) break;
  }
  return ST_OK;
}

}  // namespace

namespace {

// The captured chunk for these launch arguments, captured now if the cached
// one was made for others.  Capture runs on the context's own capture stream
// (the context stream may be the null stream, which cannot be captured); the
// graph is launched on the context stream.  A failed capture switches graphs
// off for the context (the eager launches give the same results).
template <class F>
int ensure_pcg_graph(pbr_ctx* c, int nb, const LayoutRef* L, const cplx* const* b,
                     cplx* const* x, double shift, int chunk, F&& iterate) {
  pbr_ctx::PcgGraph& G = c->pcg_graph;
  bool same = G.exec && G.nb == nb && G.chunk == chunk && G.shift == shift &&
              G.mat_gen == c->mat_gen;
  for (int t = 0; same && t < nb; ++t)
    same = G.blocks[t] == L[t].block && G.slots[t] == L[t].slot && G.b[t] == b[t] &&
           G.x[t] == x[t] && G.kap[t][0] == L[t].kappa[0] && G.kap[t][1] == L[t].kappa[1] &&
           G.kap[t][2] == L[t].kappa[2];
  if (same) return ST_OK;
  if (G.exec) (void)hipGraphExecDestroy(G.exec);
  if (G.graph) (void)hipGraphDestroy(G.graph);
  G = pbr_ctx::PcgGraph();
  if (!c->cap_stream &&
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    c->graphs_broken = true;
    return ST_OK;
  }
  const hipStream_t saved = c->stream;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->graphs_broken = true;
    return ST_OK;
  }
  c->stream = c->cap_stream;
  const int s = iterate(chunk);
  c->stream = saved;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  if (s != ST_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess || !graph ||
      hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    G.exec = nullptr;
    c->graphs_broken = true;
    (void)hipGetLastError();
    return ST_OK;
  }
  G.graph = graph;
  G.nb = nb;
  G.chunk = chunk;
  G.shift = shift;
  G.mat_gen = c->mat_gen;
  for (int t = 0; t < nb; ++t) {
    G.blocks[t] = L[t].block;
    G.slots[t] = L[t].slot;
    for (int l = 0; l < 3; ++l) G.kap[t][l] = L[t].kappa[l];
    G.b[t] = b[t];
    G.x[t] = x[t];
  }
  return ST_OK;
}

}  // namespace

// PCG for (A + shift M) x_t = b_t in nb layouts of one kind at once: every
// launch of an iteration covers all of them, and a layout that has converged
// drops out through its device flag.  Results per layout in iters[] / conv[];
// returns ST_ENOCONV on a breakdown.
int pcg_solve_batch(pbr_ctx* c, int nb, const LayoutRef* L, double shift,
                    const cplx* const* b, cplx* const* x, const pbr_opts& o, int* iters,
                    int* conv) {
  if (nb < 1 || nb > PBR_MAX_BATCH) {
    c->set_error("batch of 1 to PBR_MAX_BATCH layouts expected");
    return ST_EINVAL;
  }
  for (int t = 0; t < nb; ++t) PBR_TRY(ensure_work(c, L[t].slot, L[t].block));
  PcgScalars hs[NSTATE];
  if (!o.precond) {
    for (int t = 0; t < nb; ++t)
      PBR_TRY(pcg_plain(c, L[t].slot, L[t].block, L[t].kappa, shift, b[t], x[t], o));
  } else {
    // fused iteration: matvec (+ (p, q) partials) and five preconditioner passes
    // that also update r, p and x (x in the last pass, with the old p) and
    // finish the CG scalars on the device
    const Geo g = make_geo(c, L[0].block, L[0].kappa);
    PcgStep P[PBR_MAX_BATCH];
    ApplyLayout AL[PBR_MAX_BATCH];
    for (int t = 0; t < nb; ++t) {
      LayoutWork& W = c->wk(L[t].slot, L[t].block);
      P[t].slot = L[t].slot;
      P[t].block = L[t].block;
      for (int l = 0; l < 3; ++l) P[t].kappa[l] = L[t].kappa[l];
      P[t].st = W.st;
      P[t].tol2 = o.tol_inner * o.tol_inner;
      P[t].x = x[t];
      P[t].r = W.r;
      P[t].p = W.p;
      P[t].q = W.q;
      P[t].b = b[t];
      P[t].z = W.z;
      P[t].pout = W.p;
      P[t].part_pq = W.ppart;
      P[t].part_rr = W.ppart + W.pcap;
      P[t].part_rz = W.ppart + 2 * W.pcap;
      P[t].part_cap = W.pcap;
      P[t].init = 1;
      const Geo gt = make_geo(c, L[t].block, L[t].kappa);
      AL[t].block = L[t].block;
      for (int l = 0; l < 3; ++l) AL[t].ph[l] = gt.ph[l];
      AL[t].x = W.p;
      AL[t].y = W.q;
      AL[t].st = W.st;
      AL[t].part = W.ppart;
    }
    PBR_TRY(launch_pcg_precond_batch(c, nb, P, shift));
    for (int t = 0; t < nb; ++t) P[t].init = 0;
    const int chunk = o.check_every > 0 ? o.check_every : 10;
    auto iterate = [&](int count) -> int {
      for (int it = 0; it < count; ++it) {
        int npq = 0;
        PBR_TRY(launch_apply_batch(c, g, nb, AL, shift, P[0].part_cap, &npq));
        for (int t = 0; t < nb; ++t) P[t].n_pq = npq;
        PBR_TRY(launch_pcg_precond_batch(c, nb, P, shift));
      }
      return ST_OK;
    };
    // let the stencil's autotuner see this batch before a graph freezes the
    // launch (q = A p of the initial p; the first iteration recomputes it)
    if (o.graphs && !c->graphs_broken && !apply_tuned(c, g, nb)) {
      int npq = 0;
      PBR_TRY(launch_apply_batch(c, g, nb, AL, shift, P[0].part_cap, &npq));
    }
    // The first host check comes after about as many iterations as the previous
    // solve of this context needed (solves along a path need nearly the same
    // number); iterations past convergence are no-ops on the device (every pass
    // returns once the layout's flag is set), so only the host waits change.
    int done_iters = 0;
    bool first = true;
    for (;;) {
      const int todo = std::min(chunk, o.maxit_inner - done_iters);
      if (todo <= 0) break;
      int burst = 1;
      if (first && todo == chunk)
        burst = std::max(1, std::min((c->pcg_hint - 2 * chunk) / chunk,
                                     (o.maxit_inner - done_iters) / chunk));
      first = false;
      if (o.graphs && todo == chunk && !c->graphs_broken)
        PBR_TRY(ensure_pcg_graph(c, nb, L, b, x, shift, chunk, iterate));
      for (int rep = 0; rep < burst; ++rep) {
        if (o.graphs && todo == chunk && !c->graphs_broken)
          PBR_HIP(c, hipGraphLaunch(c->pcg_graph.exec, c->stream));
        else
          PBR_TRY(iterate(todo));
      }
      PBR_TRY(read_states(c, hs));
      bool all = true;
      done_iters = 0;
      for (int t = 0; t < nb; ++t) {
        const PcgScalars& h = hs[state_index(L[t].slot, L[t].block)];
        done_iters = std::max(done_iters, h.iters);
        all = all && h.done;
      }
      if (all) break;
    }
    c->pcg_hint = done_iters;
    // the x update of an iteration that ended at the convergence test
    PcgScalars* sts[PBR_MAX_BATCH];
    const cplx* ps[PBR_MAX_BATCH];
    for (int t = 0; t < nb; ++t) {
      sts[t] = P[t].st;
      ps[t] = P[t].p;
    }
    PBR_TRY(pcg_fix_x(c, c->stream, 3 * c->layout_nodes(L[0].block), nb, sts, x, ps));
  }
  PBR_TRY(read_states(c, hs));
  int status = ST_OK;
  for (int t = 0; t < nb; ++t) {
    const PcgScalars& h = hs[state_index(L[t].slot, L[t].block)];
    iters[t] = h.iters;
    conv[t] = (h.done == 1) ? 1 : 0;
    if (h.done == 2) {
      c->set_error("PCG breakdown: (p, (A + shift M) p) <= 0");
      status = ST_ENOCONV;
    }
  }
  return status;
}

int pcg_solve(pbr_ctx* c, int block, const double kappa[3], double shift, const cplx* b, cplx* x,
              const pbr_opts& o, int* iters, int* conv) {
  LayoutRef L;
  L.block = block;
  for (int l = 0; l < 3; ++l) L.kappa[l] = kappa[l];
  return pcg_solve_batch(c, 1, &L, shift, &b, &x, o, iters, conv);
}

namespace {

struct OpCounters {
  int applies = 0, pcg_total = 0, pcg_max = 0, matvecs = 0, pcg_fail = 0;
};

// State of one thick-restart Lanczos run (one layout).  The runs of a batch
// advance in lockstep: each step is one shift-invert application, done for all
// active runs by one batched PCG.
struct LanczosRun {
  int slot = 0, block = -1, nev = 0, m = 0, ldh = 0;
  double kappa[3] = {0, 0, 0};
  bool gamma = false;
  long N = 0, n3 = 0, ld = 0;
  int n_zero = 0;
  int j = 0, restarts = 0, nconv = 0;
  bool exhausted = false, done = false;
  int status = ST_OK;
  std::vector<zc> H;  // column-major, leading dimension ldh
  std::vector<double> beta, theta, Yr, Hd, hbuf;
  std::vector<int> order;
  OpCounters cnt;
  std::chrono::steady_clock::time_point t0;
};

// Rayleigh-Ritz on the leading mm x mm block of H; the Ritz residuals of the
// Krylov-Schur relation are |b_last * (last entry of the Ritz vector)|.
int lz_ritz(pbr_ctx* c, LanczosRun& R, int mm, double bl, const pbr_opts& o) {
  for (int jj = 0; jj < mm; ++jj)
    for (int ii = 0; ii < mm; ++ii) {
      R.Hd[2 * ((size_t)jj * mm + ii)] = R.H[(size_t)jj * R.ldh + ii].real();
      R.Hd[2 * ((size_t)jj * mm + ii) + 1] = R.H[(size_t)jj * R.ldh + ii].imag();
    }
  if (pbr_host_heev(mm, R.Hd.data(), R.theta.data(), R.Yr.data()) != 0) {
    c->set_error("Rayleigh-Ritz eigensolver failed");
    return ST_EINVAL;
  }
  R.order.resize(mm);
  for (int i = 0; i < mm; ++i) R.order[i] = mm - 1 - i;  // largest mu first
  R.nconv = 0;
  for (int i = 0; i < std::min(R.nev, mm); ++i) {
    const int col = R.order[i];
    const zc ylast(R.Yr[2 * ((size_t)col * mm + (mm - 1))],
                   R.Yr[2 * ((size_t)col * mm + (mm - 1)) + 1]);
    if (bl * std::abs(ylast) <= o.tol * std::abs(R.theta[col]))
      ++R.nconv;
    else
      break;
  }
  return ST_OK;
}

int lz_start(pbr_ctx* c, LanczosRun& R, const LayoutRef& L, int nev, const pbr_opts& o) {
  R.t0 = std::chrono::steady_clock::now();
  const int block = L.block;
  const double* kappa = L.kappa;
  PBR_TRY(ensure_work(c, L.slot, block));
  LayoutWork& W = c->wk(L.slot, block);
  R.slot = L.slot;
  for (int l = 0; l < 3; ++l) R.kappa[l] = kappa[l];
  R.block = block;
  R.nev = nev;
  R.N = W.N;
  R.n3 = 3 * W.N;
  R.ld = R.n3;
  R.gamma = is_gamma(kappa);
  if (R.gamma) {
    PBR_TRY(ensure_null_fields(c, L.slot, block));
    R.n_zero = 3 * W.nf;
  }
  const long dim_eff = R.n3 - R.n_zero;
  if (nev < 1 || nev >= dim_eff) {
    c->set_error("nev must satisfy 1 <= nev < dim - n_zero");
    return ST_EINVAL;
  }
  int m = o.ncv > 0 ? o.ncv : std::max(2 * nev + 10, 20);
  if (m > dim_eff) m = (int)dim_eff;
  if (m < nev + 1) m = nev + 1;
  if ((long)m * m > SMALL_CPLX || m > 90) {
    c->set_error("Krylov basis size ncv too large (at most 90)");
    return ST_EINVAL;
  }
  R.m = R.ldh = m;
  PBR_TRY(ensure_basis(c, W, m + 1));
  R.H.assign((size_t)m * m, zc(0, 0));
  R.beta.assign(m, 0.0);
  R.theta.assign(m, 0.0);
  R.Yr.assign(2 * (size_t)m * m, 0.0);
  R.Hd.assign(2 * (size_t)m * m, 0.0);
  R.hbuf.assign(4 * m + 8, 0.0);
  // start vector: random, or the sum of the Ritz vectors a finished run of this
  // layout kind left in a work area plus a random part of half that norm
  const hipStream_t SO = c->stream;
  int st_err;
  PBR_TRY(vec_random(c, SO, R.n3, (unsigned long long)(o.seed * 7919 + 17 + block), W.U));
  if (o.warm_start && L.warm_slot >= 0) {
    LayoutWork& S = c->wk(L.warm_slot, block);
    const int nw = std::min(S.ritz_n, S.ucols);
    if (nw > 0 && S.U2 && S.N == W.N) {
      const double rn = vnorm(c, W, W.U, &st_err);
      PBR_TRY(st_err);
      PBR_TRY(vec_scale(c, SO, R.n3, W.U, 0.5 * std::sqrt((double)nw) / rn));
      PBR_TRY(upload_small(c, W.small, std::vector<zc>(nw, zc(-1.0, 0.0))));
      PBR_TRY(gemv_sub(c, SO, R.n3, nw, S.U2, R.ld, W.small, W.U));  // U += sum of columns
    }
  }
  W.ritz_n = 0;  // this run now uses the work area
  if (R.gamma) PBR_TRY(project_null(c, W, W.U));
  const double nrm = vnorm(c, W, W.U, &st_err);
  PBR_TRY(st_err);
  PBR_TRY(vec_scale(c, SO, R.n3, W.U, 1.0 / nrm));
  R.j = 0;
  return ST_OK;
}

// Continue run R after W.w = Op u_j: orthogonalise, extend H, test convergence,
// restart when the basis is full.
int lz_step(pbr_ctx* c, LanczosRun& R, const pbr_opts& o) {
  LayoutWork& W = c->wk(R.slot, R.block);
  const hipStream_t SO = c->stream;
  const int j = R.j;
  const long n3 = R.n3, ld = R.ld;
  int st_err;
  if (R.gamma) PBR_TRY(project_null(c, W, W.w));
  // classical Gram-Schmidt, twice
  std::vector<zc> h(j + 1, zc(0, 0));
  for (int pass = 0; pass < 2; ++pass) {
    PBR_TRY(multi_dot_async(c, SO, n3, j + 1, W.U, ld, W.w, W.part, W.dscal));
    PBR_TRY(readback(c, W.dscal, R.hbuf.data(), 2 * (j + 1)));
    std::vector<zc> hp(j + 1);
    for (int i = 0; i <= j; ++i) {
      hp[i] = zc(R.hbuf[2 * i], R.hbuf[2 * i + 1]);
      h[i] += hp[i];
    }
    PBR_TRY(upload_small(c, W.small, hp));
    PBR_TRY(gemv_sub(c, SO, n3, j + 1, W.U, ld, W.small, W.w));
  }
  if (R.gamma) PBR_TRY(project_null(c, W, W.w));
  const double b = vnorm(c, W, W.w, &st_err);
  PBR_TRY(st_err);
  const int ldh = R.ldh;
  for (int i = 0; i <= j; ++i) {
    R.H[(size_t)j * ldh + i] = h[i];
    R.H[(size_t)i * ldh + j] = std::conj(h[i]);
  }
  R.H[(size_t)j * ldh + j] = zc(h[j].real(), 0.0);
  R.beta[j] = b;
  if (j + 1 < R.m) {
    R.H[(size_t)j * ldh + (j + 1)] = b;
    R.H[(size_t)(j + 1) * ldh + j] = b;
  }
  cplx* un = W.U + (long)(j + 1) * ld;
  if (b > 1e-14 * std::abs(h[j]) && b > 0.0) {
    PBR_TRY(vec_copy(c, SO, n3, W.w, un));
    PBR_TRY(vec_scale(c, SO, n3, un, 1.0 / b));
  } else {
    // invariant subspace: the Ritz values of H are exact
    R.beta[j] = 0.0;
    if (j + 1 < R.m) {
      R.H[(size_t)j * ldh + (j + 1)] = 0.0;
      R.H[(size_t)(j + 1) * ldh + j] = 0.0;
    }
    R.m = j + 1;
    R.exhausted = true;
    PBR_TRY(lz_ritz(c, R, R.m, 0.0, o));
    R.done = true;
    return ST_OK;
  }
  // convergence test after every step once the basis exceeds nev: stop as soon
  // as the wanted Ritz pairs have converged
  if (j + 1 > R.nev && j + 1 < R.m) {
    PBR_TRY(lz_ritz(c, R, j + 1, R.beta[j], o));
    if (R.nconv >= R.nev) {
      R.m = j + 1;
      R.done = true;
      return ST_OK;
    }
  }
  if (j + 1 < R.m) {
    R.j = j + 1;
    return ST_OK;
  }
  // basis full: Rayleigh-Ritz, then stop or thick-restart with kk Ritz vectors
  const int m = R.m;
  PBR_TRY(lz_ritz(c, R, m, R.beta[m - 1], o));
  if (R.nconv >= R.nev || R.restarts >= o.maxit_outer) {
    R.done = true;
    return ST_OK;
  }
  int kk = R.nev + (m - R.nev) / 2;
  if (kk >= m) kk = m - 1;
  std::vector<zc> Yk((size_t)m * kk);
  for (int cc = 0; cc < kk; ++cc)
    for (int r = 0; r < m; ++r) {
      const int col = R.order[cc];
      Yk[(size_t)cc * m + r] =
          zc(R.Yr[2 * ((size_t)col * m + r)], R.Yr[2 * ((size_t)col * m + r) + 1]);
    }
  PBR_TRY(upload_small(c, W.small, Yk));
  PBR_TRY(combine(c, SO, n3, m, kk, W.U, ld, W.small, W.U2, ld));
  PBR_TRY(vec_copy(c, SO, n3, W.U + (long)m * ld, W.U2 + (long)kk * ld));
  std::swap(W.U, W.U2);
  std::fill(R.H.begin(), R.H.end(), zc(0, 0));
  for (int i = 0; i < kk; ++i) R.H[(size_t)i * ldh + i] = R.theta[R.order[i]];
  R.j = kk;
  ++R.restarts;
  return ST_OK;
}

// Ritz vectors of the nev largest mu, final Rayleigh quotients and residuals
// with the exact operator, eigenvalues ascending.
int lz_finish(pbr_ctx* c, LanczosRun& R, double* evals, cplx* evecs_dev, pbr_stats* st) {
  const double* kappa = R.kappa;
  LayoutWork& W = c->wk(R.slot, R.block);
  DevMaterial& M = c->material(R.block);
  const hipStream_t SO = c->stream;
  const long N = R.N, n3 = R.n3, ld = R.ld;
  const int m = R.m;
  const int nout = std::min(R.nev, m);
  std::vector<zc> Yk((size_t)m * nout);
  for (int cc = 0; cc < nout; ++cc)
    for (int r = 0; r < m; ++r) {
      const int col = R.order[cc];
      Yk[(size_t)cc * m + r] =
          zc(R.Yr[2 * ((size_t)col * m + r)], R.Yr[2 * ((size_t)col * m + r) + 1]);
    }
  PBR_TRY(upload_small(c, W.small, Yk));
  PBR_TRY(combine(c, SO, n3, m, nout, W.U, ld, W.small, W.U2, ld));
  const Geo g = make_geo(c, R.block, kappa);
  std::vector<std::pair<double, int>> lam(nout);
  double max_res = 0.0;
  for (int i = 0; i < nout; ++i) {
    cplx* u = W.U2 + (long)i * ld;
    if (R.gamma) PBR_TRY(project_null(c, W, u));
    // v = M^{-1/2} u  -> W.t ;  y = A v -> W.q
    PBR_TRY(vec_diag_scale(c, SO, N, M.isrho, u, W.t));
    PBR_TRY(launch_apply(c, g, R.block, 0.0, W.t, W.q));
    R.cnt.matvecs += 1;
    double vals[3];
    PBR_TRY(dot_real_async(c, SO, n3, W.t, W.q, W.part, W.dscal));       // v^H A v
    PBR_TRY(dot_real_async(c, SO, n3, u, u, W.part, W.dscal + 1));        // v^H M v
    PBR_TRY(dot_real_async(c, SO, n3, W.q, W.q, W.part, W.dscal + 2));    // |Av|^2
    PBR_TRY(readback(c, W.dscal, vals, 3));
    const double l = vals[0] / vals[1];
    // r = A v - l M v = y - l * srho .* u
    PBR_TRY(vec_resid(c, SO, N, l, M.srho, u, W.q, W.z));
    double rr;
    PBR_TRY(dot_real_async(c, SO, n3, W.z, W.z, W.part, W.dscal));
    PBR_TRY(readback(c, W.dscal, &rr, 1));
    // |M v| = |srho .* u|
    PBR_TRY(vec_diag_scale(c, SO, N, M.srho, u, W.z));
    double mv;
    PBR_TRY(dot_real_async(c, SO, n3, W.z, W.z, W.part, W.dscal));
    PBR_TRY(readback(c, W.dscal, &mv, 1));
    const double denom = std::sqrt(vals[2]) + std::fabs(l) * std::sqrt(mv);
    const double rel = denom > 0 ? std::sqrt(rr) / denom : 0.0;
    max_res = std::max(max_res, rel);
    lam[i] = {l, i};
    if (evecs_dev) {
      // M-normalised eigenvector: v / sqrt(v^H M v)
      PBR_TRY(vec_copy(c, SO, n3, W.t, evecs_dev + (long)i * n3));
      PBR_TRY(vec_scale(c, SO, n3, evecs_dev + (long)i * n3, 1.0 / std::sqrt(vals[1])));
    }
  }
  std::sort(lam.begin(), lam.end());
  for (int i = 0; i < nout; ++i) evals[i] = lam[i].first;
  // U2 keeps the Ritz vectors for a later warm start (unless reused below)
  W.ritz_n = evecs_dev ? 0 : nout;
  if (evecs_dev) {
    // reorder columns to ascending eigenvalue
    bool sorted = true;
    for (int i = 0; i < nout; ++i) sorted = sorted && lam[i].second == i;
    if (!sorted) {
      for (int i = 0; i < nout; ++i)
        PBR_TRY(vec_copy(c, SO, n3, evecs_dev + (long)lam[i].second * n3, W.U2 + (long)i * ld));
      for (int i = 0; i < nout; ++i)
        PBR_TRY(vec_copy(c, SO, n3, W.U2 + (long)i * ld, evecs_dev + (long)i * n3));
    }
  }
  PBR_HIP(c, hipStreamSynchronize(SO));
  if (st) {
    st->outer_iters += R.restarts;
    st->op_applies += R.cnt.applies;
    st->pcg_iters_total += R.cnt.pcg_total;
    st->pcg_iters_max = std::max(st->pcg_iters_max, R.cnt.pcg_max);
    st->matvecs += R.cnt.matvecs;
    st->n_zero += R.n_zero;
    st->converged += std::min(R.nconv, R.nev);
    st->pcg_avg = st->op_applies ? (double)st->pcg_iters_total / st->op_applies : 0.0;
    st->max_rel_resid = std::max(st->max_rel_resid, max_res);
    st->seconds +=
        std::chrono::duration<double>(std::chrono::steady_clock::now() - R.t0).count();
  }
  if (R.nconv < R.nev && !R.exhausted) {
    c->set_error("outer Krylov iteration did not converge within maxit_outer restarts");
    return ST_ENOCONV;
  }
  return ST_OK;
}

// One shift-invert application w = M^{1/2} (A + shift M)^{-1} M^{1/2} u_j for
// every active run, as one batched PCG.
int op_apply_batch(pbr_ctx* c, double shift, const pbr_opts& o, LanczosRun* const* R, int na) {
  LayoutRef L[PBR_MAX_BATCH];
  int its[PBR_MAX_BATCH], conv[PBR_MAX_BATCH];
  const cplx* b[PBR_MAX_BATCH];
  cplx* x[PBR_MAX_BATCH];
  for (int t = 0; t < na; ++t) {
    LayoutWork& W = c->wk(R[t]->slot, R[t]->block);
    const DevMaterial& M = c->material(R[t]->block);
    L[t].slot = R[t]->slot;
    L[t].block = R[t]->block;
    for (int l = 0; l < 3; ++l) L[t].kappa[l] = R[t]->kappa[l];
    PBR_TRY(vec_diag_scale(c, c->stream, W.N, M.srho, W.U + (long)R[t]->j * R[t]->ld, W.b));
    b[t] = W.b;
    x[t] = W.t;
  }
  const int s = pcg_solve_batch(c, na, L, shift, b, x, o, its, conv);
  if (s != ST_OK && s != ST_ENOCONV) return s;
  for (int t = 0; t < na; ++t) {
    LayoutWork& W = c->wk(R[t]->slot, R[t]->block);
    const DevMaterial& M = c->material(R[t]->block);
    OpCounters& k = R[t]->cnt;
    k.applies += 1;
    k.pcg_total += its[t];
    k.pcg_max = std::max(k.pcg_max, its[t]);
    k.matvecs += its[t];
    if (!conv[t]) k.pcg_fail += 1;
    PBR_TRY(vec_diag_scale(c, c->stream, W.N, M.srho, W.t, W.w));
  }
  return ST_OK;
}

}  // namespace

// Lanczos runs for nb layouts of one kind in lockstep (one batched PCG per
// step).  Per-layout results go to evals[t], evecs_dev[t] (may be null) and
// st[t]; rc[t] is each run's status.  Returns the first hard error, else OK.
int lanczos_batch(pbr_ctx* c, int nb, const LayoutRef* L, const int* nev, double shift,
                  const pbr_opts& o, double* const* evals, cplx* const* evecs_dev,
                  pbr_stats* st, int* rc) {
  if (nb < 1 || nb > PBR_MAX_BATCH) {
    c->set_error("batch of 1 to PBR_MAX_BATCH layouts expected");
    return ST_EINVAL;
  }
  std::vector<LanczosRun> R(nb);
  for (int t = 0; t < nb; ++t) PBR_TRY(lz_start(c, R[t], L[t], nev[t], o));
  for (;;) {
    LanczosRun* act[PBR_MAX_BATCH];
    int na = 0;
    for (int t = 0; t < nb; ++t)
      if (!R[t].done) act[na++] = &R[t];
    if (!na) break;
    PBR_TRY(op_apply_batch(c, shift, o, act, na));
    for (int t = 0; t < na; ++t) PBR_TRY(lz_step(c, *act[t], o));
  }
  for (int t = 0; t < nb; ++t) {
    rc[t] = lz_finish(c, R[t], evals[t], evecs_dev ? evecs_dev[t] : nullptr,
                      st ? &st[t] : nullptr);
    if (rc[t] != ST_OK && rc[t] != ST_ENOCONV) return rc[t];
  }
  return ST_OK;
}

int lanczos_eigs(pbr_ctx* c, const double kappa[3], int block, int nev, double shift,
                 const pbr_opts& o, double* evals, cplx* evecs_dev, pbr_stats* st) {
  int rc = ST_OK;
  LayoutRef L;
  L.block = block;
  for (int l = 0; l < 3; ++l) L.kappa[l] = kappa[l];
  PBR_TRY(lanczos_batch(c, 1, &L, &nev, shift, o, &evals, &evecs_dev, st, &rc));
  return rc;
}

namespace {

void add_stats(pbr_stats* acc, const pbr_stats& one) {
  acc->outer_iters += one.outer_iters;
  acc->op_applies += one.op_applies;
  acc->pcg_iters_total += one.pcg_iters_total;
  acc->pcg_iters_max = std::max(acc->pcg_iters_max, one.pcg_iters_max);
  acc->matvecs += one.matvecs;
  acc->n_zero += one.n_zero;
  acc->converged += one.converged;
  acc->max_rel_resid = std::max(acc->max_rel_resid, one.max_rel_resid);
  acc->pcg_avg = acc->op_applies ? (double)acc->pcg_iters_total / acc->op_applies : 0.0;
}

}  // namespace

// Lowest nev eigenvalues of the full pencil at each of nk wave vectors from the
// four blocks (Corollary 4.2): each block is asked for ceil(nev/4) + 1 values
// (the full spectrum's near-fourfold clusters put one member in each block, so a
// block rarely holds more than ceil(nev/4) of the lowest nev); a block
// whose largest computed value lies below the merged nev-th value may hide
// smaller ones that were not computed, so it is solved again with more values
// until no block is flagged.  Up to PBR_KSLOTS k-points are solved at once, all
// their pending (k, block) runs in lockstep (opts.concurrent; else one run after
// another).  evals: nk x nev; stats summed over the k-points (nev_block of the
// last one).
int merged_path(pbr_ctx* c, int nk, const double* kappas, int nev, double shift,
                const pbr_opts& o, double* evals, pbr_stats* st, cplx* evecs_dev,
                int* blocks_out) {
  const long dimb = 3 * (c->n / 4);
  int status = ST_OK;
  int last_nev_b[4] = {0, 0, 0, 0};
  const bool want_vecs = evecs_dev != nullptr;
  if (want_vecs && (nk != 1 || !blocks_out)) {
    c->set_error("merged eigenvectors: one wave vector and a block index array expected");
    return ST_EINVAL;
  }
  // eigenvectors of each block's latest solve (want_vecs only), freed on return
  struct BlockVecs {
    cplx* v[4] = {nullptr, nullptr, nullptr, nullptr};
    int cap[4] = {0, 0, 0, 0};
    ~BlockVecs() {
      for (cplx* p : v) dev_free(p);
    }
  } bv;
  for (int k0 = 0; k0 < nk; k0 += PBR_KSLOTS) {
    const int gk = std::min(PBR_KSLOTS, nk - k0);
    int nev_b[PBR_KSLOTS][4], need[PBR_KSLOTS], flagged[PBR_KSLOTS] = {0, 0, 0, 0};
    std::vector<double> vals[PBR_KSLOTS][4];
    for (int q = 0; q < gk; ++q) {
      const double* kap = kappas + 3 * (k0 + q);
      const int nz = is_gamma(kap) ? 3 : 0;
      for (int b = 0; b < 4; ++b)
        nev_b[q][b] = (int)std::min<long>((nev + 3) / 4 + 1, dimb - nz - 1);
      need[q] = 0xF;
    }
    for (int round = 0; round < 8; ++round) {
      LayoutRef L[PBR_MAX_BATCH];
      int nevs[PBR_MAX_BATCH], rc[PBR_MAX_BATCH], qk[PBR_MAX_BATCH];
      double* ev[PBR_MAX_BATCH];
      cplx* evp[PBR_MAX_BATCH] = {};
      pbr_stats part[PBR_MAX_BATCH];
      int np = 0;
      for (int q = 0; q < gk; ++q)
        for (int b = 0; b < 4; ++b) {
          if (!(need[q] & (1 << b))) continue;
          vals[q][b].assign(nev_b[q][b], 0.0);
          L[np].slot = q;
          L[np].block = b;
          for (int l = 0; l < 3; ++l) L[np].kappa[l] = kappas[3 * (k0 + q) + l];
          // warm start: a re-solve from its own Ritz vectors, a first solve from
          // those of the last wave vector of the previous group (same block)
          L[np].warm_slot = round > 0 ? q : (k0 > 0 ? PBR_KSLOTS - 1 : -1);
          nevs[np] = nev_b[q][b];
          ev[np] = vals[q][b].data();
          if (want_vecs) {
            if (bv.cap[b] < nev_b[q][b]) {
              dev_free(bv.v[b]);
              bv.v[b] = nullptr;
              bv.cap[b] = 0;
              PBR_TRY(dev_alloc(c, (void**)&bv.v[b], sizeof(cplx) * dimb * nev_b[q][b]));
              bv.cap[b] = nev_b[q][b];
            }
            evp[np] = bv.v[b];
          }
          qk[np] = q;
          rc[np] = ST_OK;
          ++np;
        }
      if (!np) break;
      std::memset(part, 0, sizeof(part));
      if (o.concurrent) {
        PBR_TRY(lanczos_batch(c, np, L, nevs, shift, o, ev, want_vecs ? evp : nullptr, part,
                              rc));
      } else {
        for (int t = 0; t < np; ++t)
          PBR_TRY(lanczos_batch(c, 1, L + t, nevs + t, shift, o, ev + t,
                                want_vecs ? evp + t : nullptr, part + t, rc + t));
      }
      for (int t = 0; t < np; ++t) {
        if (st) add_stats(st, part[t]);
        if (rc[t] == ST_ENOCONV) status = ST_ENOCONV;
      }
      (void)qk;
      for (int q = 0; q < gk; ++q) {
        const double* vp[4] = {vals[q][0].data(), vals[q][1].data(), vals[q][2].data(),
                               vals[q][3].data()};
        std::vector<double> merged(nev);
        const int mask = pbr_host_merge(nev, nev_b[q], vp, merged.data());
        if (mask < 0) {
          c->set_error("block merge failed: fewer eigenvalues than requested");
          return ST_EINVAL;
        }
        for (int t = 0; t < nev; ++t) evals[(long)(k0 + q) * nev + t] = merged[t];
        const double* kap = kappas + 3 * (k0 + q);
        const int nz = is_gamma(kap) ? 3 : 0;
        need[q] = 0;
        flagged[q] = mask;
        for (int b = 0; b < 4; ++b)
          if (mask & (1 << b)) {
            const int nb =
                (int)std::min<long>(nev_b[q][b] + std::max(4, nev_b[q][b] / 2), dimb - nz - 1);
            if (nb > nev_b[q][b]) {
              nev_b[q][b] = nb;
              need[q] |= 1 << b;
            }
          }
      }
    }
    // A block still flagged after the last round (or whose eigenpair count
    // cannot grow further) may hide values below the merged cut: the merged
    // values of that wave vector are not certified.
    for (int q = 0; q < gk; ++q)
      if (flagged[q]) {
        c->set_error("block merge not certified at path point " + std::to_string(k0 + q) +
                     ": a block's largest computed eigenvalue stays below the merged nev-th "
                     "value");
        status = ST_ENOCONV;
      }
    for (int b = 0; b < 4; ++b) last_nev_b[b] = nev_b[gk - 1][b];
    if (want_vecs) {
      // the nev lowest of the union in ascending order (ties: lower block, then
      // lower index first), each with its block and its block-layout eigenvector
      std::vector<std::pair<double, std::pair<int, int>>> all;
      for (int b = 0; b < 4; ++b)
        for (int i = 0; i < nev_b[0][b]; ++i) all.push_back({vals[0][b][i], {b, i}});
      std::sort(all.begin(), all.end());
      for (int t = 0; t < nev; ++t) {
        const int b = all[t].second.first, i = all[t].second.second;
        blocks_out[t] = b;
        PBR_HIP(c, hipMemcpyAsync(evecs_dev + (long)t * dimb, bv.v[b] + (long)i * dimb,
                                  sizeof(cplx) * dimb, hipMemcpyDeviceToDevice, c->stream));
      }
      PBR_HIP(c, hipStreamSynchronize(c->stream));
    }
  }
  if (st) {
    for (int b = 0; b < 4; ++b) st->nev_block[b] = last_nev_b[b];
    // Gamma null modes once per k-point (re-solved blocks are not counted twice)
    st->n_zero = 0;
    for (int q = 0; q < nk; ++q)
      if (is_gamma(kappas + 3 * q)) st->n_zero += 12;
  }
  return status;
}

int merged_eigs(pbr_ctx* c, const double kappa[3], int nev, double shift, const pbr_opts& o,
                double* evals, pbr_stats* st, cplx* evecs_dev, int* blocks_out) {
  return merged_path(c, 1, kappa, nev, shift, o, evals, st, evecs_dev, blocks_out);
}

// Full-space eigenvalues at nk wave vectors, up to PBR_KSLOTS in lockstep.
int full_path(pbr_ctx* c, int nk, const double* kappas, int nev, double shift,
              const pbr_opts& o, double* evals, pbr_stats* st) {
  int status = ST_OK;
  // groups of PBR_KSLOTS wave vectors whether or not they run in lockstep, so the
  // warm starts (and hence the results) are the same both ways
  for (int k0 = 0; k0 < nk; k0 += PBR_KSLOTS) {
    const int gk = std::min(PBR_KSLOTS, nk - k0);
    LayoutRef L[PBR_KSLOTS];
    int nevs[PBR_KSLOTS], rc[PBR_KSLOTS];
    double* ev[PBR_KSLOTS];
    pbr_stats part[PBR_KSLOTS];
    std::memset(part, 0, sizeof(part));
    for (int q = 0; q < gk; ++q) {
      L[q].slot = q;
      L[q].block = -1;
      for (int l = 0; l < 3; ++l) L[q].kappa[l] = kappas[3 * (k0 + q) + l];
      L[q].warm_slot = k0 > 0 ? PBR_KSLOTS - 1 : -1;
      nevs[q] = nev;
      ev[q] = evals + (long)(k0 + q) * nev;
      rc[q] = ST_OK;
    }
    if (o.concurrent) {
      PBR_TRY(lanczos_batch(c, gk, L, nevs, shift, o, ev, nullptr, part, rc));
    } else {
      for (int q = 0; q < gk; ++q)
        PBR_TRY(lanczos_batch(c, 1, L + q, nevs + q, shift, o, ev + q, nullptr, part + q,
                              rc + q));
    }
    for (int q = 0; q < gk; ++q) {
      if (st) add_stats(st, part[q]);
      if (rc[q] == ST_ENOCONV) status = ST_ENOCONV;
    }
  }
  return status;
}

extern "C" int pbr_host_merge(int nev, const int nev_b[4], const double* const vals[4],
                              double* merged) {
  if (nev < 1 || !nev_b || !vals || !merged) return -1;
  std::vector<double> all;
  for (int b = 0; b < 4; ++b) {
    if (nev_b[b] < 0 || (nev_b[b] > 0 && !vals[b])) return -1;
    for (int t = 0; t < nev_b[b]; ++t) all.push_back(vals[b][t]);
  }
  if ((int)all.size() < nev) return -1;
  std::sort(all.begin(), all.end());
  for (int t = 0; t < nev; ++t) merged[t] = all[t];
  const double cut = all[nev - 1];
  int mask = 0;
  for (int b = 0; b < 4; ++b)
    if (nev_b[b] > 0 && vals[b][nev_b[b] - 1] < cut) mask |= 1 << b;
  return mask;
}
