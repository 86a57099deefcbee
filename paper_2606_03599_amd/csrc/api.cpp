// C interface of libpbr (declared in include/pbr.h): argument validation,
// host/device marshalling and dispatch to the kernels and solver drivers.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pbr.h"
#include "blas.hpp"
#include "context.hpp"

namespace {

thread_local std::string g_create_error;

bool finite_all(const double* p, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

int check_block(pbr_ctx* c, int block) {
  if (block < -1 || block > 3) {
    c->set_error("block must be -1 (full space) or 0..3");
    return ST_EINVAL;
  }
  if (block >= 0 && !c->even) {
    c->set_error("parity blocks need even n1, n2, n3 (Theorem 4.1)");
    return ST_EODDGRID;
  }
  return ST_OK;
}

int check_kappa(pbr_ctx* c, const double* k) {
  if (!k || !std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2])) {
    c->set_error("kappa must be 3 finite doubles");
    return ST_EINVAL;
  }
  return ST_OK;
}

int check_material(pbr_ctx* c) {
  if (!c->have_material) {
    c->set_error("pbr_set_material has not been called");
    return ST_ESTATE;
  }
  return ST_OK;
}

pbr_opts resolve_opts(const pbr_opts* o) {
  pbr_opts r;
  pbr_opts_default(&r);
  if (o) r = *o;
  return r;
}

int check_opts(pbr_ctx* c, const pbr_opts& o) {
  if (!(o.tol > 0) || !(o.tol_inner > 0) || o.maxit_outer < 0 || o.maxit_inner < 1 ||
      o.ncv < 0 || (o.precond != 0 && o.precond != 1) || o.check_every < 0 ||
      (o.concurrent != 0 && o.concurrent != 1) || (o.graphs != 0 && o.graphs != 1) ||
      (o.warm_start != 0 && o.warm_start != 1)) {
    c->set_error("invalid pbr_opts");
    return ST_EINVAL;
  }
  return ST_OK;
}

// Stage a (possibly host) vector of n3 complex into device memory.
struct Staged {
  pbr_ctx* c;
  cplx* dev = nullptr;
  bool owned = false;
  ~Staged() {
    if (owned) dev_free(dev);
  }
};

int stage_in(pbr_ctx* c, const void* p, long n3, int on_device, Staged& s) {
  s.c = c;
  if (on_device) {
    s.dev = (cplx*)p;
    return ST_OK;
  }
  PBR_TRY(dev_alloc(c, (void**)&s.dev, sizeof(cplx) * n3));
  s.owned = true;
  if (p)
    PBR_HIP(c, hipMemcpyAsync(s.dev, p, sizeof(cplx) * n3, hipMemcpyHostToDevice, c->stream));
  return ST_OK;
}

int stage_out(pbr_ctx* c, Staged& s, void* p, long n3, int on_device) {
  if (on_device) return ST_OK;
  PBR_HIP(c, hipMemcpyAsync(p, s.dev, sizeof(cplx) * n3, hipMemcpyDeviceToHost, c->stream));
  PBR_HIP(c, hipStreamSynchronize(c->stream));
  return ST_OK;
}

int finish_host(pbr_ctx* c, int on_device) {
  if (!on_device) PBR_HIP(c, hipStreamSynchronize(c->stream));
  return ST_OK;
}


}  // namespace

Geo make_geo(const pbr_ctx* c, int block, const double kappa[3]) {
  Geo g;
  geo_layout(g, c->n1, c->n2, c->n3, block);
  for (int l = 0; l < 3; ++l) {
    const double phi = 2.0 * M_PI * kappa[l];
    g.ph[l] = mk(std::cos(phi), std::sin(phi));
  }
  for (int m = 0; m < 3; ++m)
    for (int d = 0; d < 5; ++d) g.cf[m][d] = c->cf[m][d];
  return g;
}

extern "C" {

void pbr_opts_default(pbr_opts* o) {
  if (!o) return;
  o->tol = 1e-12;
  o->tol_inner = 1e-12;
  o->maxit_outer = 300;
  o->maxit_inner = 200;
  o->ncv = 0;
  o->precond = 1;
  o->check_every = 0;
  o->seed = 1;
  o->concurrent = 1;
  o->graphs = 1;
  o->warm_start = 1;
}

pbr_status pbr_create(pbr_ctx** out, int n1, int n2, int n3, const double* A_lat, int hip_device,
                      void* hip_stream) {
  if (!out) {
    g_create_error = "out is NULL";
    return PBR_EINVAL;
  }
  *out = nullptr;
  if (n1 < 1 || n2 < 1 || n3 < 1 || (long)n1 * n2 * n3 > (1L << 31)) {
    g_create_error = "grid sizes must be >= 1 (and n1*n2*n3 < 2^31)";
    return PBR_EINVAL;
  }
  double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (A_lat) std::memcpy(A, A_lat, sizeof(A));
  // A column-major: A(r,c) = A[c*3 + r]
  auto Ae = [&](int r, int cc) { return A[cc * 3 + r]; };
  const double det = Ae(0, 0) * (Ae(1, 1) * Ae(2, 2) - Ae(1, 2) * Ae(2, 1)) -
                     Ae(0, 1) * (Ae(1, 0) * Ae(2, 2) - Ae(1, 2) * Ae(2, 0)) +
                     Ae(0, 2) * (Ae(1, 0) * Ae(2, 1) - Ae(1, 1) * Ae(2, 0));
  if (!std::isfinite(det) || std::fabs(det) < 1e-300) {
    g_create_error = "A_lat is singular";
    return PBR_EINVAL;
  }
  pbr_ctx* c = new (std::nothrow) pbr_ctx();
  if (!c) {
    g_create_error = "out of host memory";
    return PBR_ENOMEM;
  }
  c->n1 = n1;
  c->n2 = n2;
  c->n3 = n3;
  c->n = (long)n1 * n2 * n3;
  c->even = (n1 % 2 == 0) && (n2 % 2 == 0) && (n3 % 2 == 0);
  std::memcpy(c->Alat, A, sizeof(A));
  // inverse by cofactors: Ainv(r,c) = cof(c,r)/det, stored row-major
  double inv[3][3];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) {
      const int r1 = (cc + 1) % 3, r2 = (cc + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
      inv[r][cc] = (Ae(r1, c1) * Ae(r2, c2) - Ae(r1, c2) * Ae(r2, c1)) / det;
    }
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) c->Ainv[r * 3 + cc] = inv[r][cc];
  // reduced stencil of D~_s (Eq. 3.11 with c_s = h_d/(4 h_s), h_s = 1/n_s):
  // D~_1 = (n1/4) sum_l S_dl - n1 I, D~_2 = (n2/4)(S1+S2-S3-S4), D~_3 = (n3/4)(S1-S2+S3-S4)
  double red[3][5] = {{-(double)n1, n1 / 4.0, n1 / 4.0, n1 / 4.0, n1 / 4.0},
                      {0.0, n2 / 4.0, n2 / 4.0, -n2 / 4.0, -n2 / 4.0},
                      {0.0, n3 / 4.0, -n3 / 4.0, n3 / 4.0, -n3 / 4.0}};
  // Cartesian D'_m = sum_s (A_lat^-1)_{sm} D~_s (Eq. 3.13 without the factor -i)
  for (int m = 0; m < 3; ++m)
    for (int d = 0; d < 5; ++d) {
      double s = 0.0;
      for (int sd = 0; sd < 3; ++sd) s += inv[sd][m] * red[sd][d];
      c->cf[m][d] = s;
    }
  c->device = hip_device;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) {
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreate(&c->stream);
      c->own_stream = (e == hipSuccess);
    }
  }
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount,
                                               hip_device);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->hpinned, sizeof(double) * PBR_PINNED);
  if (e != hipSuccess) {
    g_create_error = std::string("HIP device setup failed: ") + hipGetErrorString(e);
    if (c->hpinned) (void)hipHostFree(c->hpinned);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return PBR_EDEVICE;
  }
  if (scratch_init(c) != ST_OK || preload_kernels(c) != ST_OK) {
    g_create_error = c->err;
    (void)hipHostFree(c->hpinned);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return PBR_EDEVICE;
  }
  *out = c;
  return PBR_OK;
}

void pbr_destroy(pbr_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& M : c->mat) {
    dev_free(M.Ct);
    dev_free(M.rho);
    dev_free(M.srho);
    dev_free(M.isrho);
    dev_free(M.idx);
  }
  dev_free(c->pal);
  for (auto& T : c->fft) {
    for (int l = 0; l < 3; ++l) {
      dev_free(T.twist[l]);
      dev_free(T.post[l]);
      dev_free(T.roots[l]);
    }
    for (cplx* t : T.postp) dev_free(t);
  }
  for (auto& W : c->work) {
    cplx* vs[] = {W.x, W.r, W.p, W.q, W.z, W.b, W.w, W.t, W.U, W.U2, W.small};
    for (cplx* v : vs) dev_free(v);
    dev_free(W.part);
    dev_free(W.part2);
    dev_free(W.dscal);
    dev_free(W.ppart);
    dev_free(W.Wnull);
  }
  if (c->pcg_graph.exec) (void)hipGraphExecDestroy(c->pcg_graph.exec);
  if (c->pcg_graph.graph) (void)hipGraphDestroy(c->pcg_graph.graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  dev_free(c->st_all);
  if (c->hpinned) (void)hipHostFree(c->hpinned);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

void* pbr_stream(const pbr_ctx* c) { return c ? (void*)c->stream : nullptr; }

pbr_status pbr_copy_probe(pbr_ctx* c, const void* src, void* dst, long bytes) {
  if (!c) return PBR_EINVAL;
  if (!src || !dst || bytes < 0 || bytes % 16 != 0) {
    c->set_error("copy probe: device pointers and a byte count that is a multiple of 16 expected");
    return PBR_EINVAL;
  }
  (void)hipSetDevice(c->device);
  return (pbr_status)launch_copy_probe(c, src, dst, bytes);
}

const char* pbr_last_error(const pbr_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

pbr_status pbr_set_material(pbr_ctx* c, const double* C21, const double* rho, int on_device) {
  if (!c) return PBR_EINVAL;
  if (!C21 || !rho) {
    c->set_error("C21 and rho must be non-NULL");
    return PBR_EINVAL;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    c->set_error("hipSetDevice failed");
    return PBR_EDEVICE;
  }
  const long n = c->n;
  std::vector<double> hC, hr;
  const double* pC = C21;
  const double* pr = rho;
  if (on_device) {
    hC.resize((size_t)21 * n);
    hr.resize(n);
    if (hipMemcpy(hC.data(), C21, sizeof(double) * 21 * n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hr.data(), rho, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) {
      c->set_error("reading device material failed");
      return PBR_EDEVICE;
    }
    pC = hC.data();
    pr = hr.data();
  }
  if (!finite_all(pC, 21 * n) || !finite_all(pr, n)) {
    c->set_error("material contains NaN or Inf");
    return PBR_EINVAL;
  }
  double cmax = 0.0, rsum = 0.0;
  double csum[21] = {};
  for (long x = 0; x < n; ++x) {
    if (!(pr[x] > 0.0)) {
      c->set_error("rho must be > 0 at every node");
      return PBR_EINVAL;
    }
    rsum += pr[x];
    for (int q = 0; q < 21; ++q) {
      cmax = std::max(cmax, std::fabs(pC[(size_t)x * 21 + q]));
      csum[q] += pC[(size_t)x * 21 + q];
    }
  }
  int s = upload_material(c, pC, pr);
  if (s != ST_OK) return (pbr_status)s;
  c->rho_host.assign(pr, pr + n);
  c->Cmax = cmax;
  for (int q = 0; q < 21; ++q) c->Cref[q] = csum[q] / (double)n;
  c->rho_ref = rsum / (double)n;
  // Gamma null fields depend on rho
  for (auto& W : c->work) {
    dev_free(W.Wnull);
    W.Wnull = nullptr;
    W.nf = 0;
  }
  c->have_material = true;
  ++c->mat_gen;
  return PBR_OK;
}

pbr_status pbr_set_reference(pbr_ctx* c, const double* C21_ref, double rho_ref) {
  if (!c) return PBR_EINVAL;
  if (!C21_ref || !finite_all(C21_ref, 21) || !(rho_ref > 0.0) || !std::isfinite(rho_ref)) {
    c->set_error("reference material must be 21 finite values and rho_ref > 0");
    return PBR_EINVAL;
  }
  std::memcpy(c->Cref, C21_ref, sizeof(c->Cref));
  c->rho_ref = rho_ref;
  ++c->mat_gen;
  return PBR_OK;
}

pbr_status pbr_set_palette(pbr_ctx* c, int enable) {
  if (!c) return PBR_EINVAL;
  if (enable != 0 && enable != 1) {
    c->set_error("enable must be 0 or 1");
    return PBR_EINVAL;
  }
  if (c->use_palette != (enable == 1)) {
    c->use_palette = enable == 1;
    ++c->mat_gen;
  }
  return PBR_OK;
}

pbr_status pbr_set_stencil_shape(pbr_ctx* c, int ti, int tj) {
  if (!c) return PBR_EINVAL;
  const bool ok = (ti == 0 && tj == 0) || (ti == 16 && (tj == 13 || tj == 11));
  if (!ok) {
    c->set_error("stencil shape must be 0 x 0 (autotuned), 16 x 13 or 16 x 11");
    return PBR_EINVAL;
  }
  if (c->pin_ti != ti || c->pin_tj != tj) {
    c->pin_ti = ti;
    c->pin_tj = tj;
    ++c->mat_gen;  // captured PCG graphs hold the old launch shape
  }
  return PBR_OK;
}

pbr_status pbr_set_solve_width(pbr_ctx* c, int bi) {
  if (!c) return PBR_EINVAL;
  if (bi != 0 && bi != 8 && bi != 16 && bi != 32) {
    c->set_error("mode-solve width must be 0 (autotuned), 8, 16 or 32");
    return PBR_EINVAL;
  }
  if (c->pin_bi != bi) {
    c->pin_bi = bi;
    ++c->mat_gen;  // captured PCG graphs hold the old launch shape
  }
  return PBR_OK;
}

pbr_status pbr_set_precond_passes(pbr_ctx* c, int passes) {
  if (!c) return PBR_EINVAL;
  if (passes != 0 && passes != 3 && passes != 5) {
    c->set_error("precond passes: 0 (automatic), 3 or 5 expected");
    return PBR_EINVAL;
  }
  c->precond_passes = passes;
  c->mat_gen += 1;  // captured PCG graphs hold the old pass structure
  return PBR_OK;
}

int pbr_material_palette(const pbr_ctx* c) {
  if (!c || !c->have_material) return -1;
  return c->use_palette ? c->npal : 0;
}

double pbr_default_shift(const pbr_ctx* c) {
  if (!c || !c->have_material) return -1.0;
  return 0.30 * c->Cmax;
}

long pbr_block_dim(const pbr_ctx* c, int block) {
  if (!c || block < -1 || block > 3) return -1;
  if (block >= 0 && !c->even) return -1;
  return 3 * c->layout_nodes(block);
}

pbr_status pbr_block_gather(pbr_ctx* c, int block, const void* full, void* blk, int on_device) {
  if (!c) return PBR_EINVAL;
  int s = check_block(c, block);
  if (s == ST_OK && block < 0) {
    c->set_error("gather needs a block in 0..3");
    s = ST_EINVAL;
  }
  if (s == ST_OK && (!full || !blk)) {
    c->set_error("NULL vector");
    s = ST_EINVAL;
  }
  if (s != ST_OK) return (pbr_status)s;
  hipSetDevice(c->device);
  Staged f, b;
  if ((s = stage_in(c, full, 3 * c->n, on_device, f)) != ST_OK) return (pbr_status)s;
  if ((s = stage_in(c, nullptr, 3 * (c->n / 4), on_device, b)) != ST_OK) return (pbr_status)s;
  if (on_device) b.dev = (cplx*)blk;
  if ((s = layout_gather(c, block, f.dev, b.dev)) != ST_OK) return (pbr_status)s;
  return (pbr_status)stage_out(c, b, blk, 3 * (c->n / 4), on_device);
}

pbr_status pbr_block_scatter(pbr_ctx* c, int block, const void* blk, void* full, int on_device) {
  if (!c) return PBR_EINVAL;
  int s = check_block(c, block);
  if (s == ST_OK && block < 0) {
    c->set_error("scatter needs a block in 0..3");
    s = ST_EINVAL;
  }
  if (s == ST_OK && (!full || !blk)) {
    c->set_error("NULL vector");
    s = ST_EINVAL;
  }
  if (s != ST_OK) return (pbr_status)s;
  hipSetDevice(c->device);
  Staged b, f;
  if ((s = stage_in(c, blk, 3 * (c->n / 4), on_device, b)) != ST_OK) return (pbr_status)s;
  // scatter leaves the other entries untouched: stage the existing full vector
  if ((s = stage_in(c, full, 3 * c->n, on_device, f)) != ST_OK) return (pbr_status)s;
  if ((s = layout_scatter(c, block, b.dev, f.dev)) != ST_OK) return (pbr_status)s;
  return (pbr_status)stage_out(c, f, full, 3 * c->n, on_device);
}

pbr_status pbr_eig_grad(pbr_ctx* c, const double kappa[3], int block, int nvec,
                        const double* lambda, const double* weight, const void* evecs,
                        int evecs_on_device, double* gC21, double* grho, int grad_on_device) {
  if (!c) return PBR_EINVAL;
  int st = check_block(c, block);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK && (nvec < 1 || !lambda || !weight || !evecs || !gC21 || !grho)) {
    c->set_error("nvec >= 1 and non-NULL lambda, weight, evecs, gC21, grho required");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  const long n3 = 3 * c->layout_nodes(block);
  Staged sv;
  if ((st = stage_in(c, evecs, n3 * nvec, evecs_on_device, sv)) != ST_OK) return (pbr_status)st;
  double* dC = grad_on_device ? gC21 : nullptr;  // dev_alloc fills null pointers only
  double* dr = grad_on_device ? grho : nullptr;
  const size_t bC = sizeof(double) * 21 * (size_t)c->n, br = sizeof(double) * (size_t)c->n;
  if (!grad_on_device) {
    if ((st = dev_alloc(c, (void**)&dC, bC)) != ST_OK) return (pbr_status)st;
    if ((st = dev_alloc(c, (void**)&dr, br)) != ST_OK) {
      dev_free(dC);
      return (pbr_status)st;
    }
  }
  hipError_t he = hipSuccess;
  auto fail = [&](const char* msg) {
    c->set_error(std::string(msg) + ": " + hipGetErrorString(he));
    if (!grad_on_device) {
      dev_free(dC);
      dev_free(dr);
    }
    return PBR_EDEVICE;
  };
  if (!grad_on_device &&
      ((he = hipMemcpyAsync(dC, gC21, bC, hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
       (he = hipMemcpyAsync(dr, grho, br, hipMemcpyHostToDevice, c->stream)) != hipSuccess))
    return fail("copying the gradient fields to the device failed");
  const Geo g = make_geo(c, block, kappa);
  if ((st = launch_eig_grad(c, g, block, nvec, lambda, weight, sv.dev, dC, dr)) != ST_OK) {
    if (!grad_on_device) {
      dev_free(dC);
      dev_free(dr);
    }
    return (pbr_status)st;
  }
  if (!grad_on_device) {
    if ((he = hipMemcpyAsync(gC21, dC, bC, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (he = hipMemcpyAsync(grho, dr, br, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (he = hipStreamSynchronize(c->stream)) != hipSuccess)
      return fail("copying the gradient fields to the host failed");
    dev_free(dC);
    dev_free(dr);
  } else if (!evecs_on_device) {
    if ((he = hipStreamSynchronize(c->stream)) != hipSuccess) return fail("gradient launch failed");
  }
  return PBR_OK;
}

pbr_status pbr_apply_blocks(pbr_ctx* c, const double kappa[3], double s, const void* x,
                            void* y, int on_device) {
  if (!c) return PBR_EINVAL;
  int st = check_block(c, 0);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK && (!x || !y || !std::isfinite(s))) {
    c->set_error("x, y must be non-NULL and s finite");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  const long nb3 = 3 * c->layout_nodes(0);
  Staged sx, sy;
  if ((st = stage_in(c, x, 4 * nb3, on_device, sx)) != ST_OK) return (pbr_status)st;
  if ((st = stage_in(c, nullptr, 4 * nb3, on_device, sy)) != ST_OK) return (pbr_status)st;
  if (on_device) sy.dev = (cplx*)y;
  const Geo g = make_geo(c, 0, kappa);
  ApplyLayout L[4];
  for (int b = 0; b < 4; ++b) {
    L[b].block = b;
    for (int l = 0; l < 3; ++l) L[b].ph[l] = g.ph[l];
    L[b].x = sx.dev + b * nb3;
    L[b].y = sy.dev + b * nb3;
  }
  if ((st = launch_apply_batch(c, g, 4, L, s)) != ST_OK) return (pbr_status)st;
  return (pbr_status)stage_out(c, sy, y, 4 * nb3, on_device);
}

pbr_status pbr_apply(pbr_ctx* c, const double kappa[3], int block, double s, const void* x,
                     void* y, int on_device) {
  if (!c) return PBR_EINVAL;
  int st = check_block(c, block);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK && (!x || !y || !std::isfinite(s))) {
    c->set_error("x, y must be non-NULL and s finite");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  const long n3 = 3 * c->layout_nodes(block);
  Staged sx, sy;
  if ((st = stage_in(c, x, n3, on_device, sx)) != ST_OK) return (pbr_status)st;
  if ((st = stage_in(c, nullptr, n3, on_device, sy)) != ST_OK) return (pbr_status)st;
  if (on_device) sy.dev = (cplx*)y;
  const Geo g = make_geo(c, block, kappa);
  if ((st = launch_apply(c, g, block, s, sx.dev, sy.dev)) != ST_OK) return (pbr_status)st;
  return (pbr_status)stage_out(c, sy, y, n3, on_device);
}

pbr_status pbr_precond(pbr_ctx* c, const double kappa[3], int block, double shift, const void* r,
                       void* z, int on_device) {
  if (!c) return PBR_EINVAL;
  int st = check_block(c, block);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK && (!r || !z || !(shift > 0.0) || !std::isfinite(shift))) {
    c->set_error("r, z must be non-NULL and shift > 0");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  const long n3 = 3 * c->layout_nodes(block);
  Staged sr, sz;
  if ((st = stage_in(c, r, n3, on_device, sr)) != ST_OK) return (pbr_status)st;
  if ((st = stage_in(c, nullptr, n3, on_device, sz)) != ST_OK) return (pbr_status)st;
  if (on_device) sz.dev = (cplx*)z;
  if ((st = launch_precond(c, kappa, block, shift, sr.dev, sz.dev)) != ST_OK)
    return (pbr_status)st;
  return (pbr_status)stage_out(c, sz, z, n3, on_device);
}

pbr_status pbr_precond_noalloc(pbr_ctx* c, const double kappa[3], int block, double shift,
                               const void* r, void* z) {
  if (!c) return PBR_EINVAL;
  int st = check_block(c, block);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK && (!r || !z || !(shift > 0.0) || !std::isfinite(shift))) {
    c->set_error("r, z must be non-NULL device pointers and shift > 0");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  return (pbr_status)launch_precond_noalloc(c, kappa, block, shift, (const cplx*)r, (cplx*)z);
}

pbr_status pbr_solve(pbr_ctx* c, const double kappa[3], int block, double shift, const void* b,
                     void* x, const pbr_opts* opts, pbr_stats* stats, int on_device) {
  if (!c) return PBR_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  const pbr_opts o = resolve_opts(opts);
  int st = check_block(c, block);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK) st = check_opts(c, o);
  if (st == ST_OK && (!b || !x || !(shift > 0.0) || !std::isfinite(shift))) {
    c->set_error("b, x must be non-NULL and shift > 0");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  const long n3 = 3 * c->layout_nodes(block);
  Staged sb, sx;
  if ((st = stage_in(c, b, n3, on_device, sb)) != ST_OK) return (pbr_status)st;
  if ((st = stage_in(c, nullptr, n3, on_device, sx)) != ST_OK) return (pbr_status)st;
  if (on_device) sx.dev = (cplx*)x;
  int iters = 0, conv = 0;
  st = pcg_solve(c, block, kappa, shift, sb.dev, sx.dev, o, &iters, &conv);
  if (st != ST_OK && st != ST_ENOCONV) return (pbr_status)st;
  int s2 = stage_out(c, sx, x, n3, on_device);
  if (s2 != ST_OK) return (pbr_status)s2;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->op_applies = 1;
    stats->pcg_iters_total = iters;
    stats->pcg_iters_max = iters;
    stats->pcg_avg = iters;
    stats->matvecs = iters;
    stats->converged = conv;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!conv) {
    c->set_error("PCG reached maxit_inner without meeting tol_inner");
    return PBR_ENOCONV;
  }
  return PBR_OK;
}

pbr_status pbr_eigs(pbr_ctx* c, const double kappa[3], int block, int nev, double shift,
                    const pbr_opts* opts, double* evals, void* evecs, int evecs_on_device,
                    pbr_stats* stats) {
  if (!c) return PBR_EINVAL;
  const pbr_opts o = resolve_opts(opts);
  int st = check_block(c, block);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK) st = check_opts(c, o);
  if (st == ST_OK && (!evals || !std::isfinite(shift))) {
    c->set_error("evals must be non-NULL and shift finite");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  if (!(shift > 0.0)) shift = pbr_default_shift(c);
  const long n3 = 3 * c->layout_nodes(block);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  Staged ev;
  if (evecs) {
    if (evecs_on_device) {
      ev.dev = (cplx*)evecs;
    } else {
      if ((st = dev_alloc(c, (void**)&ev.dev, sizeof(cplx) * n3 * (long)std::max(nev, 1))) !=
          ST_OK)
        return (pbr_status)st;
      ev.owned = true;
    }
  }
  st = lanczos_eigs(c, kappa, block, nev, shift, o, evals, ev.dev, stats);
  if (st != ST_OK && st != ST_ENOCONV) return (pbr_status)st;
  if (evecs && !evecs_on_device) {
    if (hipMemcpyAsync(evecs, ev.dev, sizeof(cplx) * n3 * nev, hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      c->set_error("copying eigenvectors to the host failed");
      return PBR_EDEVICE;
    }
  }
  return (pbr_status)st;
}

pbr_status pbr_eigs_merged(pbr_ctx* c, const double kappa[3], int nev, double shift,
                           const pbr_opts* opts, double* evals, pbr_stats* stats) {
  if (!c) return PBR_EINVAL;
  const pbr_opts o = resolve_opts(opts);
  int st = check_block(c, 0);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK) st = check_opts(c, o);
  if (st == ST_OK && (!evals || nev < 1 || !std::isfinite(shift))) {
    c->set_error("evals must be non-NULL, nev >= 1, shift finite");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  if (!(shift > 0.0)) shift = pbr_default_shift(c);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  auto t0 = std::chrono::steady_clock::now();
  st = merged_eigs(c, kappa, nev, shift, o, evals, stats);
  if (stats)
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return (pbr_status)st;
}

pbr_status pbr_eigs_merged_vecs(pbr_ctx* c, const double kappa[3], int nev, double shift,
                                const pbr_opts* opts, double* evals, int* blocks, void* evecs,
                                int evecs_on_device, pbr_stats* stats) {
  if (!c) return PBR_EINVAL;
  const pbr_opts o = resolve_opts(opts);
  int st = check_block(c, 0);
  if (st == ST_OK) st = check_kappa(c, kappa);
  if (st == ST_OK) st = check_opts(c, o);
  if (st == ST_OK && (!evals || !blocks || !evecs || nev < 1 || !std::isfinite(shift))) {
    c->set_error("evals, blocks and evecs must be non-NULL, nev >= 1, shift finite");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  if (!(shift > 0.0)) shift = pbr_default_shift(c);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  const long n3 = 3 * c->layout_nodes(0);
  Staged ev;
  if (evecs_on_device) {
    ev.dev = (cplx*)evecs;
  } else {
    if ((st = dev_alloc(c, (void**)&ev.dev, sizeof(cplx) * n3 * (long)nev)) != ST_OK)
      return (pbr_status)st;
    ev.owned = true;
  }
  auto t0 = std::chrono::steady_clock::now();
  st = merged_eigs(c, kappa, nev, shift, o, evals, stats, ev.dev, blocks);
  if (stats)
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st != ST_OK && st != ST_ENOCONV) return (pbr_status)st;
  if (!evecs_on_device) {
    if (hipMemcpyAsync(evecs, ev.dev, sizeof(cplx) * n3 * nev, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      c->set_error("copying eigenvectors to the host failed");
      return PBR_EDEVICE;
    }
  }
  return (pbr_status)st;
}

pbr_status pbr_band_path(pbr_ctx* c, int nk, const double* kappas, int nev, int blocked,
                         double shift, const pbr_opts* opts, double* evals, pbr_stats* stats) {
  if (!c) return PBR_EINVAL;
  if (nk < 1 || !kappas || !evals || nev < 1) {
    c->set_error("nk >= 1, kappas, evals non-NULL and nev >= 1 required");
    return PBR_EINVAL;
  }
  const pbr_opts o = resolve_opts(opts);
  int st = check_block(c, blocked ? 0 : -1);
  for (int q = 0; st == ST_OK && q < nk; ++q) st = check_kappa(c, kappas + 3 * q);
  if (st == ST_OK) st = check_opts(c, o);
  if (st == ST_OK && !std::isfinite(shift)) {
    c->set_error("shift must be finite");
    st = ST_EINVAL;
  }
  if (st == ST_OK) st = check_material(c);
  if (st != ST_OK) return (pbr_status)st;
  hipSetDevice(c->device);
  if (!(shift > 0.0)) shift = pbr_default_shift(c);
  const long dim = 3 * c->layout_nodes(blocked ? 0 : -1);
  if (!blocked && nev >= dim - 12) {
    c->set_error("nev must be below the dimension minus the Gamma null modes");
    return PBR_EINVAL;
  }
  auto t0 = std::chrono::steady_clock::now();
  pbr_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  st = blocked ? merged_path(c, nk, kappas, nev, shift, o, evals, &acc)
               : full_path(c, nk, kappas, nev, shift, o, evals, &acc);
  if (st != ST_OK && st != ST_ENOCONV) return (pbr_status)st;
  acc.pcg_avg = acc.op_applies ? (double)acc.pcg_iters_total / acc.op_applies : 0.0;
  acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = acc;
  return (pbr_status)st;
}

pbr_status pbr_band_paths(int ncells, pbr_ctx* const* ctxs, const int* nk,
                          const double* const* kappas, int nev, int blocked, double shift,
                          const pbr_opts* opts, double* const* evals, pbr_stats* stats) {
  if (ncells < 1 || ncells > 64 || !ctxs || !nk || !kappas || !evals) return PBR_EINVAL;
  for (int q = 0; q < ncells; ++q) {
    if (!ctxs[q] || nk[q] < 1 || !kappas[q] || !evals[q]) return PBR_EINVAL;
    for (int r = 0; r < q; ++r) {
      if (ctxs[r] == ctxs[q] || ctxs[r]->stream == ctxs[q]->stream ||
          ctxs[r]->device != ctxs[q]->device) {
        ctxs[q]->set_error("contexts of pbr_band_paths must be distinct, on one device, "
                           "with their own streams");
        return PBR_EINVAL;
      }
    }
  }
  std::vector<pbr_status> res(ncells, PBR_OK);
  std::vector<pbr_stats> acc(ncells);
  auto run = [&](int q) {
    res[q] = pbr_band_path(ctxs[q], nk[q], kappas[q], nev, blocked, shift, opts, evals[q],
                           &acc[q]);
  };
  if (ncells == 1) {
    run(0);
  } else {
    std::vector<std::thread> th;
    th.reserve(ncells);
    for (int q = 0; q < ncells; ++q) th.emplace_back(run, q);
    for (auto& t : th) t.join();
  }
  if (stats)
    for (int q = 0; q < ncells; ++q) stats[q] = acc[q];
  for (int q = 0; q < ncells; ++q)
    if (res[q] != PBR_OK) return res[q];
  return PBR_OK;
}

}  // extern "C"
