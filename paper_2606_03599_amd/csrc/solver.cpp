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
#include <thread>
#include <vector>

#include "../../include/pbr_host.h"
#include "blas.hpp"
#include "context.hpp"

typedef std::complex<double> zc;

namespace {

constexpr int SMALL_CPLX = 8192;  // capacity of LayoutWork::small

int alloc_vec(pbr_ctx* c, cplx** p, long n3) { return dev_alloc(c, (void**)p, sizeof(cplx) * n3); }

int ensure_basis(pbr_ctx* c, LayoutWork& W, int cols) {
  if (W.ucols >= cols) return ST_OK;
  dev_free(W.U);
  dev_free(W.U2);
  W.U = W.U2 = nullptr;
  W.ucols = 0;
  PBR_TRY(alloc_vec(c, &W.U, 3 * W.N * (long)cols));
  PBR_TRY(alloc_vec(c, &W.U2, 3 * W.N * (long)cols));
  W.ucols = cols;
  return ST_OK;
}

bool is_gamma(const double k[3]) {
  for (int l = 0; l < 3; ++l)
    if (k[l] != std::round(k[l])) return false;
  return true;
}

// Read `count` doubles from device to host (synchronises the layout's stream).
int readback(pbr_ctx* c, LayoutWork& W, const double* dev, double* host, int count) {
  const hipStream_t SO = c->stream_of(W.block);
  PBR_HIP(c, hipMemcpyAsync(W.hpin, dev, sizeof(double) * count, hipMemcpyDeviceToHost, SO));
  PBR_HIP(c, hipStreamSynchronize(SO));
  for (int i = 0; i < count; ++i) host[i] = W.hpin[i];
  return ST_OK;
}

int upload_small(pbr_ctx* c, LayoutWork& W, cplx* dev, const std::vector<zc>& h) {
  if ((long)h.size() > SMALL_CPLX) {
    c->set_error("Krylov basis too large for the small-matrix buffer");
    return ST_EINVAL;
  }
  const hipStream_t SO = c->stream_of(W.block);
  for (size_t i = 0; i < h.size(); ++i) {
    W.hpin[2 * i] = h[i].real();
    W.hpin[2 * i + 1] = h[i].imag();
  }
  PBR_HIP(c, hipMemcpyAsync(dev, W.hpin, sizeof(cplx) * h.size(), hipMemcpyHostToDevice, SO));
  // the pinned staging buffer is reused by the next call: wait for the copy
  PBR_HIP(c, hipStreamSynchronize(SO));
  return ST_OK;
}

// Gamma null fields of a layout: nf real fields w_f with sum_t w_f w_g = delta_fg
// such that {sqrt(rho) chi e_alpha} = span{w_f e_alpha}: the M^{1/2} image of an
// M-orthonormal basis of N_Gamma.  Full space: chi in {1, (-1)^{i+j},
// (-1)^{i+k}, (-1)^{j+k}} (4 fields); a block: all four are +-1 on the class,
// so one field sqrt(rho)/sqrt(sum rho).
int ensure_null_fields(pbr_ctx* c, int block) {
  LayoutWork& W = c->work[block + 1];
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
  const hipStream_t SO = c->stream_of(block);
  PBR_HIP(c, hipMemcpyAsync(W.Wnull, F.data(), sizeof(double) * nf * N, hipMemcpyHostToDevice,
                            SO));
  PBR_HIP(c, hipStreamSynchronize(SO));
  W.nf = nf;
  return ST_OK;
}

int project_null(pbr_ctx* c, LayoutWork& W, cplx* v) {
  return proj_gamma(c, c->stream_of(W.block), W.N, W.nf, W.Wnull, v, W.part, W.dscal);
}

double vnorm(pbr_ctx* c, LayoutWork& W, const cplx* v, int* status) {
  double h;
  int s = dot_real_async(c, c->stream_of(W.block), 3 * W.N, v, v, W.part, W.dscal);
  if (s == ST_OK) s = readback(c, W, W.dscal, &h, 1);
  *status = s;
  return std::sqrt(std::max(h, 0.0));
}

}  // namespace

int ensure_work(pbr_ctx* c, int block) {
  LayoutWork& W = c->work[block + 1];
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
  PBR_TRY(dev_alloc(c, (void**)&W.st, sizeof(PcgScalars)));
  W.pcap = N / 128 + 4096;
  PBR_TRY(dev_alloc(c, (void**)&W.ppart, sizeof(double) * 3 * W.pcap));
  if (!W.hpin) PBR_HIP(c, hipHostMalloc((void**)&W.hpin, sizeof(double) * 32768));
  return ST_OK;
}

int pcg_solve(pbr_ctx* c, int block, const double kappa[3], double shift, const cplx* b, cplx* x,
              const pbr_opts& o, int* iters, int* conv) {
  PBR_TRY(ensure_work(c, block));
  LayoutWork& W = c->work[block + 1];
  const hipStream_t SO = c->stream_of(block);
  const long n3 = 3 * W.N;
  const Geo g = make_geo(c, block, kappa);
  const int chunk = o.check_every > 0 ? o.check_every : 10;
  int done_iters = 0;
  PcgScalars hs;
  auto read_state = [&]() -> int {
    PBR_HIP(c, hipMemcpyAsync(W.hpin, W.st, sizeof(PcgScalars), hipMemcpyDeviceToHost, SO));
    PBR_HIP(c, hipStreamSynchronize(SO));
    std::memcpy(&hs, W.hpin, sizeof(PcgScalars));
    return ST_OK;
  };
  if (o.precond) {
    // fused iteration: matvec (+ (p, q) partials) and five preconditioner passes
    // that also update x, r and p and finish the CG scalars on the device
    PcgStep P;
    P.st = W.st;
    P.tol2 = o.tol_inner * o.tol_inner;
    P.x = x;
    P.r = W.r;
    P.p = W.p;
    P.q = W.q;
    P.b = b;
    P.z = W.z;
    P.pout = W.p;
    P.part_pq = W.ppart;
    P.part_rr = W.ppart + W.pcap;
    P.part_rz = W.ppart + 2 * W.pcap;
    P.part_cap = W.pcap;
    P.init = 1;
    PBR_TRY(launch_pcg_precond(c, kappa, block, shift, P));
    P.init = 0;
    for (;;) {
      const int todo = std::min(chunk, o.maxit_inner - done_iters);
      if (todo <= 0) break;
      for (int it = 0; it < todo; ++it) {
        PBR_TRY(launch_apply(c, g, block, shift, W.p, W.q, W.st, W.ppart, W.pcap, &P.n_pq));
        PBR_TRY(launch_pcg_precond(c, kappa, block, shift, P));
      }
      PBR_TRY(read_state());
      done_iters = hs.iters;
      if (hs.done) break;
    }
  } else {
    PBR_TRY(vec_zero(c, SO, n3, x));
    PBR_TRY(vec_copy(c, SO, n3, b, W.r));
    PBR_TRY(vec_copy(c, SO, n3, W.r, W.z));
    PBR_TRY(vec_copy(c, SO, n3, W.z, W.p));
    PBR_TRY(pcg_init_async(c, SO, n3, W.r, W.z, o.tol_inner, W.part, W.part2, W.st));
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
      PBR_TRY(read_state());
      done_iters = hs.iters;
      if (hs.done) break;
    }
  }
  PBR_TRY(read_state());
  *iters = hs.iters;
  *conv = (hs.done == 1) ? 1 : 0;
  if (hs.done == 2) {
    c->set_error("PCG breakdown: (p, (A + shift M) p) <= 0");
    return ST_ENOCONV;
  }
  return ST_OK;
}

namespace {

struct OpCounters {
  int applies = 0, pcg_total = 0, pcg_max = 0, matvecs = 0, pcg_fail = 0;
};

// w = M^{1/2} (A + shift M)^{-1} M^{1/2} u
int op_apply(pbr_ctx* c, int block, const double kappa[3], double shift, const pbr_opts& o,
             const cplx* u, cplx* w, OpCounters& cnt) {
  LayoutWork& W = c->work[block + 1];
  DevMaterial& M = c->material(block);
  const hipStream_t SO = c->stream_of(block);
  PBR_TRY(vec_diag_scale(c, SO, W.N, M.srho, u, W.b));
  int it = 0, conv = 0;
  int s = pcg_solve(c, block, kappa, shift, W.b, W.t, o, &it, &conv);
  if (s != ST_OK && s != ST_ENOCONV) return s;
  cnt.applies += 1;
  cnt.pcg_total += it;
  cnt.pcg_max = std::max(cnt.pcg_max, it);
  cnt.matvecs += it;
  if (!conv) cnt.pcg_fail += 1;
  PBR_TRY(vec_diag_scale(c, SO, W.N, M.srho, W.t, w));
  return ST_OK;
}

}  // namespace

int lanczos_eigs(pbr_ctx* c, const double kappa[3], int block, int nev, double shift,
                 const pbr_opts& o, double* evals, cplx* evecs_dev, pbr_stats* st) {
  auto t0 = std::chrono::steady_clock::now();
  PBR_TRY(ensure_work(c, block));
  LayoutWork& W = c->work[block + 1];
  DevMaterial& M = c->material(block);
  const hipStream_t SO = c->stream_of(block);
  const long N = W.N, n3 = 3 * N;
  const bool gamma = is_gamma(kappa);
  int n_zero = 0;
  if (gamma) {
    PBR_TRY(ensure_null_fields(c, block));
    n_zero = 3 * W.nf;
  }
  const long dim_eff = n3 - n_zero;
  if (nev < 1 || nev >= dim_eff) {
    c->set_error("nev must satisfy 1 <= nev < dim - n_zero");
    return ST_EINVAL;
  }
  int m = o.ncv > 0 ? o.ncv : std::max(2 * nev + 10, 20);
  if (m > dim_eff) m = (int)dim_eff;
  if (m < nev + 1) m = nev + 1;
  if ((long)m * m > SMALL_CPLX || m > 120) {
    c->set_error("Krylov basis size ncv too large (at most 90)");
    return ST_EINVAL;
  }
  PBR_TRY(ensure_basis(c, W, m + 1));
  const long ld = n3;
  OpCounters cnt;
  int st_err;
  // start vector
  PBR_TRY(vec_random(c, SO, n3, (unsigned long long)(o.seed * 7919 + 17 + block), W.U));
  if (gamma) PBR_TRY(project_null(c, W, W.U));
  double nrm = vnorm(c, W, W.U, &st_err);
  PBR_TRY(st_err);
  PBR_TRY(vec_scale(c, SO, n3, W.U, 1.0 / nrm));

  std::vector<zc> H((size_t)m * m, zc(0, 0));  // column-major, leading dimension ldh
  const int ldh = m;
  std::vector<double> beta(m, 0.0);
  std::vector<double> theta(m);
  std::vector<double> Yr(2 * (size_t)m * m);
  std::vector<double> Hd(2 * (size_t)m * m);
  std::vector<double> hbuf(4 * m + 8);
  int j0 = 0;
  int restarts = 0;
  int nconv = 0;
  bool exhausted = false;
  std::vector<int> order;
  // Rayleigh-Ritz on the leading mm x mm block of H; the Ritz residuals of the
  // Krylov-Schur relation are |b_last * (last entry of the Ritz vector)|.
  auto ritz = [&](int mm, double bl) -> int {
    for (int jj = 0; jj < mm; ++jj)
      for (int ii = 0; ii < mm; ++ii) {
        Hd[2 * ((size_t)jj * mm + ii)] = H[(size_t)jj * ldh + ii].real();
        Hd[2 * ((size_t)jj * mm + ii) + 1] = H[(size_t)jj * ldh + ii].imag();
      }
    if (pbr_host_heev(mm, Hd.data(), theta.data(), Yr.data()) != 0) {
      c->set_error("Rayleigh-Ritz eigensolver failed");
      return ST_EINVAL;
    }
    order.resize(mm);
    for (int i = 0; i < mm; ++i) order[i] = mm - 1 - i;  // largest mu first
    nconv = 0;
    for (int i = 0; i < std::min(nev, mm); ++i) {
      const int col = order[i];
      const zc ylast(Yr[2 * ((size_t)col * mm + (mm - 1))],
                     Yr[2 * ((size_t)col * mm + (mm - 1)) + 1]);
      if (bl * std::abs(ylast) <= o.tol * std::abs(theta[col]))
        ++nconv;
      else
        break;
    }
    return ST_OK;
  };
  for (;;) {
    bool early = false;
    for (int j = j0; j < m; ++j) {
      cplx* uj = W.U + (long)j * ld;
      PBR_TRY(op_apply(c, block, kappa, shift, o, uj, W.w, cnt));
      if (gamma) PBR_TRY(project_null(c, W, W.w));
      // classical Gram-Schmidt, twice
      std::vector<zc> h(j + 1, zc(0, 0));
      for (int pass = 0; pass < 2; ++pass) {
        PBR_TRY(multi_dot_async(c, SO, n3, j + 1, W.U, ld, W.w, W.part, W.dscal));
        PBR_TRY(readback(c, W, W.dscal, hbuf.data(), 2 * (j + 1)));
        std::vector<zc> hp(j + 1);
        for (int i = 0; i <= j; ++i) {
          hp[i] = zc(hbuf[2 * i], hbuf[2 * i + 1]);
          h[i] += hp[i];
        }
        PBR_TRY(upload_small(c, W, W.small, hp));
        PBR_TRY(gemv_sub(c, SO, n3, j + 1, W.U, ld, W.small, W.w));
      }
      if (gamma) PBR_TRY(project_null(c, W, W.w));
      const double b = vnorm(c, W, W.w, &st_err);
      PBR_TRY(st_err);
      for (int i = 0; i <= j; ++i) {
        H[(size_t)j * ldh + i] = h[i];
        H[(size_t)i * ldh + j] = std::conj(h[i]);
      }
      H[(size_t)j * ldh + j] = zc(h[j].real(), 0.0);
      beta[j] = b;
      if (j + 1 < m) {
        H[(size_t)j * ldh + (j + 1)] = b;
        H[(size_t)(j + 1) * ldh + j] = b;
      }
      cplx* un = W.U + (long)(j + 1) * ld;
      if (b > 1e-14 * std::abs(h[j]) && b > 0.0) {
        PBR_TRY(vec_copy(c, SO, n3, W.w, un));
        PBR_TRY(vec_scale(c, SO, n3, un, 1.0 / b));
      } else {
        // invariant subspace: the Ritz values of H are exact
        beta[j] = 0.0;
        if (j + 1 < m) {
          H[(size_t)j * ldh + (j + 1)] = 0.0;
          H[(size_t)(j + 1) * ldh + j] = 0.0;
        }
        m = j + 1;
        exhausted = true;
        break;
      }
      // convergence test after every step once the basis exceeds nev: stop
      // as soon as the wanted Ritz pairs have converged
      if (j + 1 > nev && j + 1 < m) {
        PBR_TRY(ritz(j + 1, beta[j]));
        if (nconv >= nev) {
          m = j + 1;
          early = true;
          break;
        }
      }
    }
    if (!early) PBR_TRY(ritz(m, beta[m - 1]));
    if (nconv >= nev || exhausted || restarts >= o.maxit_outer) break;
    // thick restart: keep kk Ritz vectors
    int kk = nev + (m - nev) / 2;
    if (kk >= m) kk = m - 1;
    std::vector<zc> Yk((size_t)m * kk);
    for (int cc = 0; cc < kk; ++cc)
      for (int r = 0; r < m; ++r) {
        const int col = order[cc];
        Yk[(size_t)cc * m + r] = zc(Yr[2 * ((size_t)col * m + r)], Yr[2 * ((size_t)col * m + r) + 1]);
      }
    PBR_TRY(upload_small(c, W, W.small, Yk));
    PBR_TRY(combine(c, SO, n3, m, kk, W.U, ld, W.small, W.U2, ld));
    PBR_TRY(vec_copy(c, SO, n3, W.U + (long)m * ld, W.U2 + (long)kk * ld));
    std::swap(W.U, W.U2);
    std::fill(H.begin(), H.end(), zc(0, 0));
    for (int i = 0; i < kk; ++i) H[(size_t)i * ldh + i] = theta[order[i]];
    j0 = kk;
    ++restarts;
  }
  // Ritz vectors of the nev largest mu
  const int nout = std::min(nev, m);
  std::vector<zc> Yk((size_t)m * nout);
  for (int cc = 0; cc < nout; ++cc)
    for (int r = 0; r < m; ++r) {
      const int col = order[cc];
      Yk[(size_t)cc * m + r] = zc(Yr[2 * ((size_t)col * m + r)], Yr[2 * ((size_t)col * m + r) + 1]);
    }
  PBR_TRY(upload_small(c, W, W.small, Yk));
  PBR_TRY(combine(c, SO, n3, m, nout, W.U, ld, W.small, W.U2, ld));
  // final Rayleigh quotients and residuals with the exact operator
  const Geo g = make_geo(c, block, kappa);
  std::vector<std::pair<double, int>> lam(nout);
  double max_res = 0.0;
  for (int i = 0; i < nout; ++i) {
    cplx* u = W.U2 + (long)i * ld;
    if (gamma) PBR_TRY(project_null(c, W, u));
    // v = M^{-1/2} u  -> W.t ;  y = A v -> W.q
    PBR_TRY(vec_diag_scale(c, SO, N, M.isrho, u, W.t));
    PBR_TRY(launch_apply(c, g, block, 0.0, W.t, W.q));
    cnt.matvecs += 1;
    double vals[3];
    PBR_TRY(dot_real_async(c, SO, n3, W.t, W.q, W.part, W.dscal));       // v^H A v
    PBR_TRY(dot_real_async(c, SO, n3, u, u, W.part, W.dscal + 1));        // v^H M v
    PBR_TRY(dot_real_async(c, SO, n3, W.q, W.q, W.part, W.dscal + 2));    // |Av|^2
    PBR_TRY(readback(c, W, W.dscal, vals, 3));
    const double l = vals[0] / vals[1];
    // r = A v - l M v = y - l * srho .* u
    PBR_TRY(vec_resid(c, SO, N, l, M.srho, u, W.q, W.z));
    double rr;
    PBR_TRY(dot_real_async(c, SO, n3, W.z, W.z, W.part, W.dscal));
    PBR_TRY(readback(c, W, W.dscal, &rr, 1));
    // |M v| = |srho .* u|
    PBR_TRY(vec_diag_scale(c, SO, N, M.srho, u, W.z));
    double mv;
    PBR_TRY(dot_real_async(c, SO, n3, W.z, W.z, W.part, W.dscal));
    PBR_TRY(readback(c, W, W.dscal, &mv, 1));
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
    st->outer_iters += restarts;
    st->op_applies += cnt.applies;
    st->pcg_iters_total += cnt.pcg_total;
    st->pcg_iters_max = std::max(st->pcg_iters_max, cnt.pcg_max);
    st->matvecs += cnt.matvecs;
    st->n_zero += n_zero;
    st->converged += std::min(nconv, nev);
    st->pcg_avg = st->op_applies ? (double)st->pcg_iters_total / st->op_applies : 0.0;
    st->max_rel_resid = std::max(st->max_rel_resid, max_res);
    st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (nconv < nev && !exhausted) {
    c->set_error("outer Krylov iteration did not converge within maxit_outer restarts");
    return ST_ENOCONV;
  }
  return ST_OK;
}

namespace {

// Streams and events of the concurrent block solves (created once per context).
int ensure_block_streams(pbr_ctx* c) {
  for (int b = 0; b < 4; ++b) {
    if (!c->bstream[b]) PBR_HIP(c, hipStreamCreateWithFlags(&c->bstream[b], hipStreamNonBlocking));
    if (!c->join_ev[b])
      PBR_HIP(c, hipEventCreateWithFlags(&c->join_ev[b], hipEventDisableTiming));
  }
  if (!c->fork_ev) PBR_HIP(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  return ST_OK;
}

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

// Solve the blocks in `mask` concurrently: one host thread and one stream per
// block (the blocks share nothing but the read-only context data).  The block
// streams are ordered after everything already queued on the context stream, and
// the context stream after them on return.
int solve_blocks(pbr_ctx* c, const double kappa[3], int mask, const int nev_b[4], double shift,
                 const pbr_opts& o, std::vector<double>* vals, pbr_stats* st) {
  if (!o.concurrent) {
    int status = ST_OK;
    for (int b = 0; b < 4; ++b) {
      if (!(mask & (1 << b))) continue;
      vals[b].assign(nev_b[b], 0.0);
      pbr_stats one;
      std::memset(&one, 0, sizeof(one));
      const int s = lanczos_eigs(c, kappa, b, nev_b[b], shift, o, vals[b].data(), nullptr, &one);
      if (s != ST_OK && s != ST_ENOCONV) return s;
      if (s == ST_ENOCONV) status = ST_ENOCONV;
      if (st) add_stats(st, one);
    }
    return status;
  }
  PBR_TRY(ensure_block_streams(c));
  for (int b = 0; b < 4; ++b)
    if (mask & (1 << b)) PBR_TRY(ensure_work(c, b));
  PBR_HIP(c, hipEventRecord(c->fork_ev, c->stream));
  int rc[4] = {ST_OK, ST_OK, ST_OK, ST_OK};
  pbr_stats part[4];
  std::memset(part, 0, sizeof(part));
  std::vector<std::thread> th;
  for (int b = 0; b < 4; ++b) {
    if (!(mask & (1 << b))) continue;
    vals[b].assign(nev_b[b], 0.0);
    th.emplace_back([&, b]() {
      if (hipSetDevice(c->device) != hipSuccess ||
          hipStreamWaitEvent(c->bstream[b], c->fork_ev, 0) != hipSuccess) {
        c->set_error("could not start a block solve on its stream");
        rc[b] = ST_EDEVICE;
        return;
      }
      c->work[b + 1].stream = c->bstream[b];
      rc[b] = lanczos_eigs(c, kappa, b, nev_b[b], shift, o, vals[b].data(), nullptr, &part[b]);
      if (hipEventRecord(c->join_ev[b], c->bstream[b]) != hipSuccess) rc[b] = ST_EDEVICE;
      c->work[b + 1].stream = nullptr;
    });
  }
  for (auto& t : th) t.join();
  for (int b = 0; b < 4; ++b)
    if (mask & (1 << b)) PBR_HIP(c, hipStreamWaitEvent(c->stream, c->join_ev[b], 0));
  int status = ST_OK;
  for (int b = 0; b < 4; ++b) {
    if (!(mask & (1 << b))) continue;
    if (st) add_stats(st, part[b]);
    if (rc[b] == ST_ENOCONV && status == ST_OK) status = ST_ENOCONV;
    if (rc[b] != ST_OK && rc[b] != ST_ENOCONV) status = rc[b];
  }
  return status;
}

}  // namespace

// Lowest nev eigenvalues of the full pencil from the four blocks (Corollary 4.2):
// each block is asked for nev/4 + 4 values; a block whose largest computed value
// lies below the merged nev-th value may hide smaller ones that were not computed,
// so it is solved again with more values until no block is flagged.
int merged_eigs(pbr_ctx* c, const double kappa[3], int nev, double shift, const pbr_opts& o,
                double* evals, pbr_stats* st) {
  int nev_b[4];
  std::vector<double> vals[4];
  const long dimb = 3 * (c->n / 4);
  const int nz = is_gamma(kappa) ? 3 : 0;
  auto cap = [&](int v) { return (int)std::min<long>(v, dimb - nz - 1); };
  for (int b = 0; b < 4; ++b) nev_b[b] = cap((nev + 3) / 4 + 4);
  int need = 0xF;
  int status = ST_OK;
  for (int round = 0; round < 8 && need; ++round) {
    const int s = solve_blocks(c, kappa, need, nev_b, shift, o, vals, st);
    if (s == ST_ENOCONV)
      status = ST_ENOCONV;
    else if (s != ST_OK)
      return s;
    const double* vp[4] = {vals[0].data(), vals[1].data(), vals[2].data(), vals[3].data()};
    std::vector<double> merged(nev);
    const int mask = pbr_host_merge(nev, nev_b, vp, merged.data());
    if (mask < 0) {
      c->set_error("block merge failed: fewer eigenvalues than requested");
      return ST_EINVAL;
    }
    for (int t = 0; t < nev; ++t) evals[t] = merged[t];
    need = 0;
    for (int b = 0; b < 4; ++b)
      if (mask & (1 << b)) {
        const int nb = cap(nev_b[b] + std::max(4, nev_b[b] / 2));
        if (nb > nev_b[b]) {
          nev_b[b] = nb;
          need |= 1 << b;
        }
      }
  }
  if (st) {
    for (int b = 0; b < 4; ++b) st->nev_block[b] = nev_b[b];
    st->n_zero = 4 * nz;  // re-solved blocks are not counted twice
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
