// Matrix-free application of A_h(k) + s M_h = B_h C_h B_h^H + s M_h (Sec. 6.1):
// strains from the velocity at a node and its four backward diagonal
// neighbours (B^H), the nodewise 6x6 Voigt stiffness (C), then the divergence
// from the stress at the node and its four forward neighbours (B).
//
// With D'_m = sum_s (A_lat^-1)_{sm} D~_s the factors -i of Eq. 3.12 cancel in
// B C B^H, so everything is written with the real stencil D'_m = sum_d cf[m][d] S_d:
//   G_{m,a}(z) = (D'_m^H v_a)(z) = sum_d cf[m][d] v_a(z - d)
//   eps = [G11, G22, G33, G32+G23, G31+G13, G21+G12]          (rows of B^H)
//   tau = C(z) eps,   S = stress tensor of tau (S11=t1, S22=t2, S33=t3,
//                                               S23=t4, S13=t5, S12=t6)
//   y_a(x) = sum_d sum_m cf[m][d] S_{m,a}(x + d) + s rho(x) v_a(x)   (rows of B)
//
// Kernel organisation (one fused pass, HBM-bound):
//  * a work-group owns a TI x TJ tile of the (i, j) plane of the layout box and
//    streams through a chunk of planes k in [k0, k1); with TI x TJ = 16 x 13
//    the own lanes and the ring lanes (below) fill four waves, one per SIMD, so
//    a lane may hold up to 512 registers;
//  * the velocity is staged in LDS once per plane for the tile and the ring its
//    backward neighbours reach, in a ring of four planes; the loads of plane
//    s+3 are issued at the top of step s into one of two alternating register
//    sets and staged at the end of step s+1.  Staging multiplies every value by
//    the Bloch phase of its (possibly out-of-box) position, i.e. it stores the
//    extended field v(x + n_l e_l) = e^{i phi_l} v(x) of Eq. 3.2, so no later
//    step needs wrap or phase logic;
//  * the stiffness (21 entries) and rho of a plane come from the tiled layout
//    of DevMaterial::Ct (22 x 16 doubles contiguous per row run), loaded two
//    planes ahead into two alternating register sets: the set of plane s+2 is
//    refilled right after the stress of plane s has consumed it;
//  * palette form (a material with at most PBR_PAL_MAX distinct rows): the
//    same kernel reads instead one byte per node (its row), two planes ahead,
//    and takes the row's 22 doubles from a copy of the palette in LDS when the
//    stress needs them.  With the stiffness stream gone the kernel waits on
//    LDS, barriers and instruction latency rather than HBM, so this variant
//    uses a 16 x 11 tile (73 KB of LDS plus the palette) and a 256-register
//    budget, and two work-groups share a CU;
//  * for each plane s, tau is formed once per node of the tile plus the ring its
//    forward neighbours reach (i+1 column, j-1 / j+TJ rows) -- one lane per
//    position -- from the staged velocity and the stiffness, and staged in LDS;
//    the shift term s rho x of an output node is added at the same time;
//  * every output node adds the contributions of plane s to three rolling
//    accumulators (planes s-1, s, s+1: a forward step changes k by -1, 0 or +1)
//    and writes plane s-1, now complete;
//  * ring positions no output of the tile reaches (parity-dependent in a block
//    layout, where a step changes y2 by 0 or w2(i)) are skipped;
//  * tiles are numbered so that consecutive tiles go to one XCD, keeping the
//    ring re-reads of C and x in that XCD's L2; the chunk length is autotuned
//    per (batch size, box) among the best candidates of a cost model;
//  * the (x, y) partials of the fused PCG are per tile and pair of planes, so
//    no result depends on the chunking;
//  * all global accesses are buffer loads/stores with 32-bit offsets (one
//    descriptor per array, scalar plane offsets).
#include <algorithm>
#include <vector>

#include "blas.hpp"
#include "context.hpp"
#include "reduce.hpp"

namespace {

// One layout of a batched launch (the parity blocks of one grid share the box
// shape and differ in their class bits, material and vectors).
struct ApplyBlock {
  const cplx* x;
  cplx* y;
  const double* Ct;      // stiffness and rho tiles of the layout (DevMaterial::Ct)
  const unsigned char* idx;  // palette row of each node (DevMaterial::idx), palette form
  const PcgScalars* st;  // optional: this block's work-groups return once st->done != 0
  double* part;          // optional: per-work-group partials of Re(x^H y)
  int a, c;              // class bits of the block (unused in the natural layout)
  cplx ph[3];            // e^{i phi_l} of this layout's wave vector
};

struct ApplyArgs {
  Geo g;
  int N;              // nodes of one layout (all offsets below fit in 32 bits)
  int ct_tiles;       // runs of PBR_CT_W nodes per row of the stiffness tiles
  int ct_bytes;       // bytes of one layout's stiffness tiles
  const double* pal;  // palette form: npal rows of 22 doubles (C21, rho)
  int npal;
  double s;
  int tiles_i, tiles_j, chunk;
  int per;            // work-groups per layout
  // Layouts that share a material (the same parity block at different wave
  // vectors) sit next to each other in b[]: group g is b[gs[g] .. gs[g+1]).
  // Work-groups are numbered (group, tile and chunk, member), so the members of
  // a group stream the same stiffness at the same time on one XCD and all but
  // the first find it in that XCD's L2.
  int ngroups;
  int gs[PBR_MAX_BATCH + 1];
  ApplyBlock b[PBR_MAX_BATCH];
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Buffer resources: one 128-bit descriptor per array, so every access is a
// 32-bit per-lane byte offset plus a wave-uniform (scalar) offset.
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ inline double ldd(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ inline cplx ldc(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(cplx, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ inline int ldb(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return (int)__builtin_amdgcn_raw_buffer_load_b8(r, voff, soff, 0);
}
__device__ inline void stc(__amdgpu_buffer_rsrc_t r, cplx v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 0);
}

// Byte offset outside every buffer: loads through it return 0 without memory
// traffic, so lanes with nothing to load run the same straight-line code.
constexpr int OOB = 0x7ffffff0;

// e^{i q phi} from e^{i phi} for any integer q (|q| > 1 only on tiny grids).
__device__ inline cplx phase_pow(cplx ph, int q) {
  cplx r = mk(1.0, 0.0);
  const cplx b = q >= 0 ? ph : cconj(ph);
  for (int t = q >= 0 ? q : -q; t > 0; --t) r = cmul(r, b);
  return r;
}

// Wrap a virtual coordinate into [0, L) and return the number of periods crossed.
__device__ inline int wrapq(int v, int L, int& q) {
  q = (v >= 0) ? v / L : -((L - 1 - v) / L);
  return v - q * L;
}

// Offsets (dj, dk) of the backward step d (1..4) from a node with first coordinate i.
__device__ inline void bwd_offsets(const Geo& g, int i, int d, int& dj, int& dk) {
  const int s2 = step_s2(d), s3 = step_s3(d);
  if (!g.blocked) {
    dj = -s2;
    dk = -s3;
  } else {
    const int w2 = 2 * ((g.a + i) & 1) - 1;
    const int w3 = 2 * ((g.a + g.c + i) & 1) - 1;
    dj = (w2 - s2) / 2;
    dk = (w3 - s3) / 2;
  }
}

// Forward offsets (e2, e3) of step d (1..4) from a node with first coordinate i.
__device__ inline void fwd_offsets(const Geo& g, int i, int d, int& e2, int& e3) {
  const int s2 = step_s2(d), s3 = step_s3(d);
  if (!g.blocked) {
    e2 = s2;
    e3 = s3;
  } else {
    const int w2 = 2 * ((g.a + i) & 1) - 1;
    const int w3 = 2 * ((g.a + g.c + i) & 1) - 1;
    e2 = (s2 + w2) / 2;
    e3 = (s3 + w3) / 2;
  }
}

// Is tau position (ii, jj) of the tile, at virtual plane s, reached by an
// output node of the tile with plane in [k0, k1)?  (self term or a forward step)
__device__ inline bool position_needed(const Geo& g, int TI, int TJ, int i0, int j0, int iend,
                                       int jend, int k0, int k1, int ii, int jj, int s) {
  const int vi = i0 + ii, vj = j0 - 1 + jj;
  if (ii < TI && jj >= 1 && jj <= TJ && vi < iend && vj < jend && s >= k0 && s < k1) return true;
  const int src_i = vi - 1;
  if (src_i < i0 || src_i >= iend) return false;
  bool need = false;
#pragma unroll
  for (int d = 1; d <= 4; ++d) {
    int e2, e3;
    fwd_offsets(g, src_i, d, e2, e3);
    const int sj = vj - e2, st = s - e3;
    need = need || (sj >= j0 && sj < jend && st >= k0 && st < k1);
  }
  return need;
}

// Voigt stress from the velocity gradient G[m][a] = (D'_m^H v_a) and the node's
// stiffness (upper triangle, row by row).
__device__ inline void stress_of_gradient(const cplx G[3][3], const double Cz[21], cplx tau[6]) {
  cplx eps[6];
  eps[0] = G[0][0];
  eps[1] = G[1][1];
  eps[2] = G[2][2];
  eps[3] = cadd(G[2][1], G[1][2]);
  eps[4] = cadd(G[2][0], G[0][2]);
  eps[5] = cadd(G[1][0], G[0][1]);
#define CIDX(r, c) ((r) <= (c) ? ((r) * 6 - ((r) * ((r)-1)) / 2 + ((c) - (r))) \
                               : ((c) * 6 - ((c) * ((c)-1)) / 2 + ((r) - (c))))
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    cplx acc = mk(0, 0);
#pragma unroll
    for (int c = 0; c < 6; ++c) acc = cfma(Cz[CIDX(r, c)], eps[c], acc);
    tau[r] = acc;
  }
#undef CIDX
}

// y_a contribution sum_m cf[m][d] S_{m,a} of the staged stress at LDS position p.
template <int NP>
__device__ inline void contrib(const Geo& g, const cplx* lds, int p, int d, cplx out[3]) {
  const cplx t0 = lds[0 * NP + p], t1 = lds[1 * NP + p], t2 = lds[2 * NP + p];
  const cplx t3 = lds[3 * NP + p], t4 = lds[4 * NP + p], t5 = lds[5 * NP + p];
  // S rows: (t0 t5 t4), (t5 t1 t3), (t4 t3 t2)
  const double c0 = g.cf[0][d], c1 = g.cf[1][d], c2 = g.cf[2][d];
  out[0] = cfma(c2, t4, cfma(c1, t5, cscale(c0, t0)));
  out[1] = cfma(c2, t3, cfma(c1, t1, cscale(c0, t5)));
  out[2] = cfma(c2, t2, cfma(c1, t3, cscale(c0, t4)));
}

__device__ inline int wslot(int v) { return v & 3; }

// Threads of a work-group for a TI x TJ tile: TI*TJ "own" lanes (one output
// column each) followed by the ring lanes (the i+1 column and the j-1 / j+TJ
// rows of the tile), rounded up to whole waves.
__host__ __device__ constexpr int tile_threads(int TI, int TJ) {
  return ((TI * TJ + (TJ + 2) + 2 * TI) + 63) / 64 * 64;
}

// Output planes per (x, y) partial of a tile; chunks are multiples of it.
constexpr int PART_G = 2;

// Work-group layout: own lanes, then ring lanes, then idle lanes up to a wave.
// Static LDS of a TI x TJ tile: four velocity planes, the stress plane and the
// reduction slots.
__host__ __device__ constexpr int stream_static_lds(int TI, int TJ) {
  return 4 * 3 * (TI + 2) * (TJ + 4) * 16 + 6 * (TI + 1) * (TJ + 2) * 16 +
         (tile_threads(TI, TJ) / 64 + 1) * 8;
}
// Waves per SIMD a variant is compiled for: a palette-form tile whose LDS lets
// two work-groups share a CU gets half the registers.
__host__ __device__ constexpr int stream_wpe(int TI, int TJ, bool PAL) {
  return PAL && 2 * (stream_static_lds(TI, TJ) + 1024) <= 160 * 1024 ? 2 : 1;
}

template <int TI, int TJ, bool PAL>
__global__ void __launch_bounds__(tile_threads(TI, TJ))
    __attribute__((amdgpu_waves_per_eu(stream_wpe(TI, TJ, PAL), stream_wpe(TI, TJ, PAL))))
    apply_stream_kernel(ApplyArgs A) {
  constexpr int PI = TI + 1, PJ = TJ + 2, NP = PI * PJ;  // tau region
  constexpr int XI = TI + 2, XJ = TJ + 4, NX = XI * XJ;  // velocity region
  constexpr int NOWN = TI * TJ;
  constexpr int NT = tile_threads(TI, TJ);
  constexpr int NH = PJ + 2 * TI;
  constexpr int XPASS = (NX + NT - 1) / NT;
  static_assert(NOWN + NH <= NT, "own and ring lanes must fit the work-group");
  __shared__ cplx tau_s[6 * NP];
  __shared__ cplx x_s[4][3 * NX];
  __shared__ double red[NT / 64 + 1];
  extern __shared__ cplx pal_s[];  // palette form: npal rows of 11 pairs (dynamic LDS)

  // XCD-aware numbering: work-groups are dealt round-robin over 8 XCDs, so
  // give each XCD a contiguous range of (layout, tile, chunk) indices.
  const int W = gridDim.x;
  const int w = blockIdx.x;
  const int per8 = W / 8, rem = W % 8;
  const int xcd = w % 8, slot = w / 8;
  const int logical =
      (xcd < rem ? xcd * (per8 + 1) : rem * (per8 + 1) + (xcd - rem) * per8) + slot;
  int grp = 0;
  while (grp + 1 < A.ngroups && logical >= A.gs[grp + 1] * A.per) ++grp;
  const int gsize = A.gs[grp + 1] - A.gs[grp];
  const int rel = logical - A.gs[grp] * A.per;
  const int local = rel / gsize;
  const int blk = A.gs[grp] + (rel - local * gsize);
  const ApplyBlock& P = A.b[blk];
  if (P.st && P.st->done) return;  // whole work-group
  Geo g = A.g;
  g.a = P.a;
  g.c = P.c;
  g.ph[0] = P.ph[0];
  g.ph[1] = P.ph[1];
  g.ph[2] = P.ph[2];
  const int L1 = g.L1, L2 = g.L2, L3 = g.L3;
  const int N = A.N;
  const __amdgpu_buffer_rsrc_t rx = rsrc(P.x, (unsigned)N * 48u);
  const __amdgpu_buffer_rsrc_t ry = rsrc(P.y, (unsigned)N * 48u);
  const __amdgpu_buffer_rsrc_t rc = rsrc(P.Ct, (unsigned)A.ct_bytes);
  const __amdgpu_buffer_rsrc_t ri = rsrc(P.idx, PAL ? (unsigned)N : 0u);
  const int cs = N * 16;
  const int ntile = A.tiles_i * A.tiles_j;
  const int tile = local % ntile;
  const int chunk = local / ntile;
  const int i0 = (tile % A.tiles_i) * TI;
  const int j0 = (tile / A.tiles_i) * TJ;
  const int k0 = chunk * A.chunk;
  const int k1 = min(k0 + A.chunk, L3);
  const int iend = min(i0 + TI, L1), jend = min(j0 + TJ, L2);
  const int tid = threadIdx.x;

  // ---- velocity staging positions of this lane (XPASS per plane) ----
  int xoff[XPASS];     // byte offset of the actual node in one component plane
  cplx xph[XPASS];     // in-plane Bloch phase of the virtual position
#pragma unroll
  for (int r = 0; r < XPASS; ++r) {
    const int p = tid + r * NT;
    const int xc = p % XI, xr = p / XI;
    int qi, qj;
    const int ai = wrapq(i0 - 1 + xc, L1, qi);
    const int aj = wrapq(j0 - 2 + xr, L2, qj);
    xoff[r] = (p < NX) ? (ai + L1 * aj) * 16 : OOB;
    xph[r] = cmul(phase_pow(g.ph[0], qi), phase_pow(g.ph[1], qj));
  }
  // loads of velocity plane v (none when !valid: the same instructions with
  // out-of-range offsets, so the number of loads in flight never depends on
  // the path taken)
  auto stage_load = [&](int v, bool valid, cplx out[XPASS][3]) {
    int qk;
    const int kk = wrapq(v, L3, qk);
    const int kb = kk * L1 * L2 * 16;
#pragma unroll
    for (int r = 0; r < XPASS; ++r)
#pragma unroll
      for (int a = 0; a < 3; ++a)
        out[r][a] = ldc(rx, (xoff[r] == OOB || !valid) ? OOB : xoff[r] + kb, a * cs);
  };
  auto stage_store = [&](int v, cplx in[XPASS][3]) {
    int qk;
    (void)wrapq(v, L3, qk);
    const cplx phk = phase_pow(g.ph[2], qk);
    cplx* dst = x_s[wslot(v)];
#pragma unroll
    for (int r = 0; r < XPASS; ++r) {
      const int p = tid + r * NT;
      if (p < NX) {
        const cplx ph = cmul(phk, xph[r]);
#pragma unroll
        for (int a = 0; a < 3; ++a) dst[a * NX + p] = cmul(ph, in[r][a]);
      }
    }
  };

  // ---- this lane's tau position ----
  const bool own = tid < NOWN;
  const int h = tid - NOWN;
  int ii, jj;
  if (own) {
    ii = tid % TI;
    jj = tid / TI + 1;
  } else {
    ii = (h < PJ) ? TI : (h < PJ + TI ? h - PJ : h - PJ - TI);
    jj = (h < PJ) ? h : (h < PJ + TI ? 0 : PJ - 1);
  }
  const bool active = own || h < NH;
  const int vi = i0 + ii, vj = j0 - 1 + jj;
  int qi0, qj0;
  const int ai = wrapq(vi, L1, qi0);
  const int aj = wrapq(vj, L2, qj0);
  const int pos = jj * PI + ii;
  // LDS velocity indices of the node and its backward neighbours, and the
  // window plane offset of each neighbour
  const int xself = (jj + 1) * XI + ii + 1;
  int xnb[4], dkn[4];
#pragma unroll
  for (int d = 1; d <= 4; ++d) {
    int dj, dk;
    bwd_offsets(g, ai, d, dj, dk);
    xnb[d - 1] = (jj + dj + 1) * XI + ii;
    dkn[d - 1] = dk;
  }
  const bool inbox_pos = own && vi < iend && vj < jend;
  // Whether this lane's tau at plane s is read by an output of the chunk: its
  // own output node (plane s itself) or a forward step from an output node of
  // the tile at plane s - e3 (e3 in {-1, 0, 1}).  The palette form takes the
  // lane's part of that test, which does not depend on s, once here as one flag
  // per e3; the dense form evaluates it per plane (position_needed), which
  // measured faster there (its register allocation is at the limit).
  bool need_m = false, need_0 = active && inbox_pos, need_p = false;  // e3 = -1, 0, +1
  if constexpr (PAL) {
    const int src_i = vi - 1;
    const bool src_ok = active && src_i >= i0 && src_i < iend;
#pragma unroll
    for (int d = 1; d <= 4; ++d) {
      int e2, e3;
      fwd_offsets(g, src_i, d, e2, e3);
      const int sj = vj - e2;
      const bool hit = src_ok && sj >= j0 && sj < jend;
      need_m = need_m || (hit && e3 < 0);
      need_0 = need_0 || (hit && e3 == 0);
      need_p = need_p || (hit && e3 > 0);
    }
  }
  auto needed_at = [&](int s) -> bool {
    if constexpr (PAL) {
      return (need_0 && s >= k0 && s < k1) || (need_p && s - 1 >= k0 && s - 1 < k1) ||
             (need_m && s + 1 >= k0 && s + 1 < k1);
    } else {
      if (!active) return false;
      if (inbox_pos && s >= k0 && s < k1) return true;
      return position_needed(g, TI, TJ, i0, j0, iend, jend, k0, k1, ii, jj, s);
    }
  };
  // stiffness (21 entries) and rho of a tau plane into one register set
  // (entry q of the node's run is q * PBR_CT_W doubles past entry 0)
  const int ct_row = (ai / PBR_CT_W) * 22 * PBR_CT_W + ai % PBR_CT_W;
  auto load_C = [&](int s, bool need, double Cz[22]) {
    int qk;
    const int kk = wrapq(s, L3, qk);
    const int o8 = need ? ((aj + L2 * kk) * A.ct_tiles * 22 * PBR_CT_W + ct_row) * 8 : OOB;
#pragma unroll
    for (int q = 0; q < 22; ++q) Cz[q] = ldd(rc, o8, q * PBR_CT_W * 8);
  };
  // palette form: the node's palette row of a tau plane (one byte), and the
  // row itself from LDS into a register set when the stress needs it
  auto load_I = [&](int s, bool need, int& I) {
    int qk;
    const int kk = wrapq(s, L3, qk);
    I = ldb(ri, need ? ai + L1 * (aj + L2 * kk) : OOB, 0);
  };
  auto fetch_pal = [&](int I, double Cz[22]) {
    const cplx* row = pal_s + min(I, A.npal - 1) * 11;
#pragma unroll
    for (int q = 0; q < 11; ++q) {
      const cplx v = row[q];
      Cz[2 * q] = v.x;
      Cz[2 * q + 1] = v.y;
    }
  };

  // ---- output (own lanes) ----
  const int io = vi, jo = vj;
  const bool out_ok = own && io < L1 && jo < L2;
  const int w2 = g.blocked ? 2 * ((g.a + io) & 1) - 1 : 0;
  const int w3p = g.blocked ? (((g.a + g.c + io) & 1) ? 1 : 0) : 0;
  const int eA = g.blocked ? (w2 > 0 ? 1 : 0) : 1;
  const int eB = g.blocked ? (w2 > 0 ? 0 : -1) : -1;
  const int pA = (jj + eA) * PI + ii + 1;
  const int pB = (jj + eB) * PI + ii + 1;

  cplx A0[3], A1[3], A2[3];  // outputs of planes s-1, s, s+1
#pragma unroll
  for (int a = 0; a < 3; ++a) A0[a] = A1[a] = A2[a] = mk(0, 0);
  // Re(x^H y) partials, one per tile and group of PART_G output planes,
  // whatever the chunking (chunks are whole groups): each lane adds its terms
  // of a group's planes in order; at the group's last plane the wave sums go to
  // red[] and thread 0 finishes the partial at the top of the next step (after
  // the barrier that ends it).  The later sum of the partials therefore does
  // not depend on the chunk length or on how many layouts share the launch.
  const bool want_part = P.part != nullptr;
  double* const part_tile =
      want_part ? P.part + (long)tile * ((L3 + PART_G - 1) / PART_G) : nullptr;
  double xyl = 0.0;  // this lane's terms of the current group
  int pend = -1;     // group whose wave sums sit in red[]
  auto finish_part = [&]() {
    if (want_part && pend >= 0 && tid == 0) {
      double v = 0.0;
      for (int w = 0; w < NT / 64; ++w) v += red[w];
      part_tile[pend] = v;
    }
  };

  // ---- prologue: velocity planes k0-2 .. k0 staged, k0+1 in registers;
  //      stiffness of tau planes k0-1 and k0 in flight ----
  //      (all of them requested together, so the start-up waits for one
  //      round trip to memory rather than one per plane)
  cplx XA[XPASS][3], XB[XPASS][3];
  bool need_a = needed_at(k0 - 1), need_b = needed_at(k0);
  double Ca[22], Cb[22];
  int Ia = 0, Ib = 0;  // palette form: rows of the two tau planes in flight
  {
    cplx X0[XPASS][3], X1[XPASS][3];
    stage_load(k0 - 2, true, X0);
    stage_load(k0 - 1, true, X1);
    stage_load(k0, true, XA);
    stage_load(k0 + 1, k0 + 1 <= k1 + 1, XB);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (PAL) {
      load_I(k0 - 1, need_a, Ia);
      load_I(k0, need_b, Ib);
      for (int e = tid; e < A.npal * 11; e += NT)
        pal_s[e] = mk(A.pal[2 * e], A.pal[2 * e + 1]);
    } else {
      load_C(k0 - 1, need_a, Ca);
      // keep the two sets in issue order: the loop's waits count on it
      __builtin_amdgcn_sched_barrier(0);
      load_C(k0, need_b, Cb);
    }
    stage_store(k0 - 2, X0);
    stage_store(k0 - 1, X1);
    stage_store(k0, XA);
  }
  // Prefetch distances: the stiffness of plane s+2 is loaded right after the
  // stress of plane s has consumed its registers (two sets alternate), and the
  // velocity of plane s+3 is loaded at the top of step s and staged at the end
  // of step s+1 (two register sets alternate), so every load has more than a
  // whole step to arrive and no step waits for loads it issued itself.
  const double shift = A.s;
  __syncthreads();

#define PBR_STEP(S_, Cuse, Iuse, need_use, Xload, Xstore)                             \
  do {                                                                                \
    const int s = (S_);                                                               \
    finish_part();                                                                    \
    stage_load(s + 3, s + 3 <= k1 + 1, Xload);                                        \
    /* ---- tau of plane s from the staged velocity ---- */                           \
    const cplx* xs0 = x_s[wslot(s)];                                                  \
    if (need_use) {                                                                   \
      if constexpr (PAL) fetch_pal(Iuse, Cuse);                                       \
      /* velocity at the node and its four backward neighbours: all fifteen LDS */    \
      /* reads are issued together, then the gradient G[m][a] = D'_m^H v_a; */        \
      /* own nodes of an output plane also take the shift term s rho x here */        \
      cplx v0[3], vb[4][3];                                                           \
_Pragma("unroll")                                                                     \
      for (int a = 0; a < 3; ++a) v0[a] = xs0[a * NX + xself];                        \
_Pragma("unroll")                                                                     \
      for (int d = 0; d < 4; ++d) {                                                   \
        const cplx* xsd = x_s[wslot(s + dkn[d])];                                     \
_Pragma("unroll")                                                                     \
        for (int a = 0; a < 3; ++a) vb[d][a] = xsd[a * NX + xnb[d]];                  \
      }                                                                               \
      if (out_ok && s >= k0 && s < k1) {                                              \
        const double sr = shift * Cuse[21];                                           \
_Pragma("unroll")                                                                     \
        for (int a = 0; a < 3; ++a) A1[a] = cfma(sr, v0[a], A1[a]);                   \
      }                                                                               \
      cplx G[3][3];                                                                   \
_Pragma("unroll")                                                                     \
      for (int a = 0; a < 3; ++a)                                                     \
_Pragma("unroll")                                                                     \
        for (int m = 0; m < 3; ++m) {                                                 \
          cplx acc = cscale(g.cf[m][0], v0[a]);                                       \
_Pragma("unroll")                                                                     \
          for (int d = 1; d <= 4; ++d) acc = cfma(g.cf[m][d], vb[d - 1][a], acc);     \
          G[m][a] = acc;                                                              \
        }                                                                             \
      cplx tau[6];                                                                    \
      stress_of_gradient(G, Cuse, tau);                                               \
_Pragma("unroll")                                                                     \
      for (int c = 0; c < 6; ++c) tau_s[c * NP + pos] = tau[c];                       \
    }                                                                                 \
    /* stiffness of plane s+2 into the registers just consumed */                    \
    need_use = (s + 2 <= k1) && needed_at(s + 2);                                     \
    if constexpr (PAL)                                                                \
      load_I(s + 2, need_use, Iuse);                                                  \
    else                                                                              \
      load_C(s + 2, need_use, Cuse);                                                  \
    __syncthreads();                                                                  \
    /* ---- consume plane s ---- */                                                   \
    const int t = s - 1; /* output plane completed in this step */                    \
    if (out_ok) {                                                                     \
      cplx c1[3], c3[3], gP[3], gM[3];                                                \
      contrib<NP>(g, tau_s, pA, 1, c1);                                               \
      contrib<NP>(g, tau_s, pB, 3, c3);                                               \
_Pragma("unroll")                                                                     \
      for (int a = 0; a < 3; ++a) gP[a] = cadd(c1[a], c3[a]);                         \
      contrib<NP>(g, tau_s, pA, 2, c1);                                               \
      contrib<NP>(g, tau_s, pB, 4, c3);                                               \
_Pragma("unroll")                                                                     \
      for (int a = 0; a < 3; ++a) gM[a] = cadd(c1[a], c3[a]);                         \
      if (s >= k0 && s < k1) {                                                        \
        const cplx t0 = tau_s[0 * NP + pos], t5 = tau_s[5 * NP + pos];                \
        const cplx t4 = tau_s[4 * NP + pos], t1 = tau_s[1 * NP + pos];                \
        const cplx t3 = tau_s[3 * NP + pos], t2 = tau_s[2 * NP + pos];                \
        const double a0 = g.cf[0][0], a1 = g.cf[1][0], a2 = g.cf[2][0];               \
        A1[0] = cadd(A1[0], cfma(a2, t4, cfma(a1, t5, cscale(a0, t0))));              \
        A1[1] = cadd(A1[1], cfma(a2, t3, cfma(a1, t1, cscale(a0, t5))));              \
        A1[2] = cadd(A1[2], cfma(a2, t2, cfma(a1, t3, cscale(a0, t4))));              \
      }                                                                               \
      /* forward steps with s3 = +1 / -1 reach plane s from output plane s - e3: */   \
      /* natural layout e3 = s3; block layout e3 = 0 or w3. */                        \
      if (!g.blocked) {                                                               \
_Pragma("unroll")                                                                     \
        for (int a = 0; a < 3; ++a) {                                                 \
          A0[a] = cadd(A0[a], gP[a]);                                                 \
          A2[a] = cadd(A2[a], gM[a]);                                                 \
        }                                                                             \
      } else if (w3p) { /* w3 = +1: s3=+1 -> e3 = +1, s3=-1 -> e3 = 0 */              \
_Pragma("unroll")                                                                     \
        for (int a = 0; a < 3; ++a) {                                                 \
          A0[a] = cadd(A0[a], gP[a]);                                                 \
          A1[a] = cadd(A1[a], gM[a]);                                                 \
        }                                                                             \
      } else { /* w3 = -1: s3=+1 -> e3 = 0, s3=-1 -> e3 = -1 */                       \
_Pragma("unroll")                                                                     \
        for (int a = 0; a < 3; ++a) {                                                 \
          A1[a] = cadd(A1[a], gP[a]);                                                 \
          A2[a] = cadd(A2[a], gM[a]);                                                 \
        }                                                                             \
      }                                                                               \
      /* ---- plane s-1 is complete: y = B C B^H x + shift rho x ---- */              \
      if (t >= k0 && t < k1) {                                                        \
        const int o = io + L1 * (jo + L2 * t);                                        \
        cplx xprev[3];                                                                \
_Pragma("unroll")                                                                     \
        for (int a = 0; a < 3; ++a) xprev[a] = x_s[wslot(t)][a * NX + xself];         \
_Pragma("unroll")                                                                     \
        for (int a = 0; a < 3; ++a) {                                                 \
          const cplx yv = A0[a];                                                      \
          stc(ry, yv, o * 16, a * cs);                                                \
          xyl = fma(xprev[a].x, yv.x, fma(xprev[a].y, yv.y, xyl));                    \
        }                                                                             \
      }                                                                               \
    }                                                                                 \
    pend = -1;                                                                        \
    if (want_part && t >= k0 && t < k1 && (t % PART_G == PART_G - 1 || t == L3 - 1)) {\
      const double wsum = wave_sum(xyl);                                              \
      if ((tid & 63) == 0) red[tid >> 6] = wsum;                                      \
      xyl = 0.0;                                                                      \
      pend = t / PART_G;                                                              \
    }                                                                                 \
    /* velocity plane s+2 (loaded a step ago) into the slot of plane s-2 */           \
    if (s + 2 <= k1 + 1) stage_store(s + 2, Xstore);                                  \
_Pragma("unroll")                                                                     \
    for (int a = 0; a < 3; ++a) {                                                     \
      A0[a] = A1[a];                                                                  \
      A1[a] = A2[a];                                                                  \
      A2[a] = mk(0, 0);                                                               \
    }                                                                                 \
    __syncthreads();                                                                  \
  } while (0)

  for (int s0 = k0 - 1; s0 <= k1; s0 += 2) {
    PBR_STEP(s0, Ca, Ia, need_a, XA, XB);
    if (s0 + 1 <= k1) PBR_STEP(s0 + 1, Cb, Ib, need_b, XB, XA);
  }
#undef PBR_STEP
  finish_part();
}

constexpr int TILE_I = 16, TILE_J = 13;
// Palette form: without the stiffness stream the kernel waits on LDS and
// barriers rather than HBM, so besides the 16 x 13 tile (one work-group per
// CU) it has a 16 x 11 tile whose LDS (73 KB plus the palette) lets two
// work-groups share a CU; the autotuner picks between them.  (An 8 x 22 tile,
// 71 KB, timed 3-5 % slower than 16 x 11 at n = 128.)
struct TileShape {
  int ti, tj;
};
constexpr TileShape PAL_SHAPES[2] = {{16, 11}, {16, 13}};
constexpr TileShape DENSE_SHAPES[1] = {{16, 13}};
constexpr int pal_lds_bytes(int npal) { return npal * 11 * 16; }

}  // namespace

// Loads this file's kernels onto the current device (see preload_kernels).
int preload_stencil(pbr_ctx* c) {
  hipFuncAttributes a;
  PBR_HIP(c, hipFuncGetAttributes(&a, reinterpret_cast<const void*>((apply_stream_kernel<16, 11, true>))));
  return ST_OK;
}

// Work split of a launch: tile shape (16 x 13; for the palette form also
// 16 x 11) and chunk length.  A tile shape fits one work-group per CU (two for
// the palette form's 16 x 11 tile when its palette is small), so a launch runs
// in ceil(work-groups / resident work-groups) rounds, each as long as its
// longest chunk plus its start-up (the two partial planes a chunk computes at
// its ends and the first loads, which nothing overlaps); per tile shape the
// model cost rounds x (chunk + 4) ranks the chunk lengths that are whole groups
// of PART_G planes (or the whole box).  The autotuner times the four best
// candidates (the two best of each shape when there are two; only the pinned
// shape's when pbr_set_stencil_shape pins one) with real launches (three in a
// row per candidate, after a round that warms the caches) the first time a
// (batch size, box, material form, pin) is seen outside stream capture, and
// keeps the fastest in the context; a candidate replaces
// the first shape's model choice only if it is 5% faster, since candidates
// often time within noise of each other and a stable choice keeps the launch
// (and its partials) the same from run to run.  During capture, or when timing
// fails, the model's choice is used.  The launches are the caller's own (same
// inputs, same outputs, rewritten).  The (x, y) partials are per tile and group
// of planes, so no result depends on the chunk; the tile shape changes how
// they are grouped, so inner products may round differently between shapes.
template <class F>
int tuned_split(pbr_ctx* c, const Geo& g, int nb, int pal, F&& launch, int* ti_out, int* tj_out,
                int* out) {
  for (const auto& e : c->stencil_tune)
    if (e.nb == nb && e.L1 == g.L1 && e.L2 == g.L2 && e.L3 == g.L3 && e.pal == pal &&
        e.pin_ti == c->pin_ti && e.pin_tj == c->pin_tj && e.chunk > 0) {
      *ti_out = e.ti;
      *tj_out = e.tj;
      *out = e.chunk;
      return ST_OK;
    }
  const TileShape* all = pal ? PAL_SHAPES : DENSE_SHAPES;
  const int nall = pal ? 2 : 1;
  // a shape pinned by pbr_set_stencil_shape that this form has
  TileShape pinned = {0, 0};
  for (int sh = 0; sh < nall; ++sh)
    if (all[sh].ti == c->pin_ti && all[sh].tj == c->pin_tj) pinned = all[sh];
  const bool is_pinned = pinned.ti > 0;
  const TileShape* shapes = is_pinned ? &pinned : all;
  const int nshapes = is_pinned ? 1 : nall;
  struct Pick {
    int ti, tj, chunk;
  };
  std::vector<Pick> pick;  // in timing order
  for (int sh = 0; sh < nshapes; ++sh) {
    const int ti = shapes[sh].ti, tj = shapes[sh].tj;
    const int lds = stream_static_lds(ti, tj) + 256 + (pal ? pal_lds_bytes(c->npal) : 0);
    const int per_cu = std::max(1, 160 * 1024 / lds);
    const int slots = std::max(1, c->cus) * per_cu;  // work-groups resident at once
    const long tiles = (long)((g.L1 + ti - 1) / ti) * ((g.L2 + tj - 1) / tj);
    std::vector<std::pair<long, int>> cand;  // (model cost, chunk)
    for (int ch = std::min(PART_G, g.L3); ch <= g.L3; ++ch) {
      if (ch % PART_G != 0 && ch != g.L3) continue;
      const long wgs = (long)nb * tiles * ((g.L3 + ch - 1) / ch);
      cand.push_back({((wgs + slots - 1) / slots) * (ch + 4), ch});
    }
    std::stable_sort(cand.begin(), cand.end(),
                     [](const std::pair<long, int>& a, const std::pair<long, int>& b) {
                       return a.first < b.first;
                     });
    const size_t keep = std::min<size_t>(nshapes == 1 ? 4 : 2, cand.size());
    for (size_t k = 0; k < keep; ++k) pick.push_back({ti, tj, cand[k].second});
  }
  *ti_out = pick[0].ti;
  *tj_out = pick[0].tj;
  *out = pick[0].chunk;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return ST_OK;
  const int ncand = (int)pick.size();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ncand > 1 && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    float best_ms = -1.0f;
    bool ok = true;
    for (int r = 0; r < 2 && ok; ++r)  // the first round also warms the caches
      for (int k = 0; k < ncand && ok; ++k) {
        ok = hipEventRecord(e0, c->stream) == hipSuccess;
        for (int rep = 0; ok && rep < (r == 1 ? 3 : 1); ++rep)
          PBR_TRY(launch(pick[k].ti, pick[k].tj, pick[k].chunk));
        ok = ok && hipEventRecord(e1, c->stream) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (ok && r == 1 && (best_ms < 0.0f || ms < 0.95f * best_ms)) {
          best_ms = ms;
          *ti_out = pick[k].ti;
          *tj_out = pick[k].tj;
          *out = pick[k].chunk;
        }
      }
    if (!ok) {
      *ti_out = pick[0].ti;
      *tj_out = pick[0].tj;
      *out = pick[0].chunk;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  auto& slot = c->stencil_tune[c->stencil_tune_next];
  c->stencil_tune_next = (c->stencil_tune_next + 1) % PBR_TUNE_SLOTS;
  slot.nb = nb;
  slot.L1 = g.L1;
  slot.L2 = g.L2;
  slot.L3 = g.L3;
  slot.pal = pal;
  slot.pin_ti = c->pin_ti;
  slot.pin_tj = c->pin_tj;
  slot.ti = *ti_out;
  slot.tj = *tj_out;
  slot.chunk = *out;
  return ST_OK;
}

// Whether the material's palette form is the one the stencil reads.
static int apply_palette(const pbr_ctx* c) { return c->use_palette && c->npal > 0 ? 1 : 0; }

bool apply_tuned(const pbr_ctx* c, const Geo& g, int nb) {
  const int pal = apply_palette(c);
  for (const auto& e : c->stencil_tune)
    if (e.nb == nb && e.L1 == g.L1 && e.L2 == g.L2 && e.L3 == g.L3 && e.pal == pal &&
        e.chunk > 0)
      return true;
  return false;
}

long apply_partials(const pbr_ctx* c, int block) {
  const long L1 = c->n1, L2 = block < 0 ? c->n2 : c->n2 / 2, L3 = block < 0 ? c->n3 : c->n3 / 2;
  long tiles = 0;
  for (const TileShape& t : PAL_SHAPES)
    tiles = std::max(tiles, ((L1 + t.ti - 1) / t.ti) * ((L2 + t.tj - 1) / t.tj));
  for (const TileShape& t : DENSE_SHAPES)
    tiles = std::max(tiles, ((L1 + t.ti - 1) / t.ti) * ((L2 + t.tj - 1) / t.tj));
  return tiles * ((L3 + PART_G - 1) / PART_G);
}

int launch_apply_batch(pbr_ctx* c, const Geo& g, int nb, const ApplyLayout* L, double s,
                       long part_cap, int* nparts) {
  if (nb < 1 || nb > PBR_MAX_BATCH) {
    c->set_error("batch of 1 to PBR_MAX_BATCH layouts expected");
    return ST_EINVAL;
  }
  const long Nl = c->layout_nodes(g.blocked ? 0 : -1);
  const int ct_tiles = (g.L1 + PBR_CT_W - 1) / PBR_CT_W;
  const long ct_len = (long)g.L3 * g.L2 * ct_tiles * 22 * PBR_CT_W;
  if (Nl * 48L >= (1L << 31) || ct_len * 8L >= (1L << 31)) {
    c->set_error("grid too large for 32-bit buffer offsets of the stencil kernel");
    return ST_EINVAL;
  }
  ApplyArgs A;
  A.g = g;
  A.N = (int)Nl;
  A.ct_tiles = ct_tiles;
  A.ct_bytes = (int)(ct_len * 8);
  const int pal = apply_palette(c);
  A.pal = c->pal;
  A.npal = c->npal;
  A.s = s;
  // (x, y) partials per layout: the most any tile shape needs
  const long np_max = apply_partials(c, g.blocked ? 0 : -1);
  // layouts ordered by material (stable), grouped by equal material
  int ord[PBR_MAX_BATCH];
  for (int t = 0; t < nb; ++t) ord[t] = t;
  std::stable_sort(ord, ord + nb, [&](int u, int v) { return L[u].block < L[v].block; });
  A.ngroups = 0;
  for (int t = 0; t < nb; ++t)
    if (t == 0 || L[ord[t]].block != L[ord[t - 1]].block) A.gs[A.ngroups++] = t;
  A.gs[A.ngroups] = nb;
  for (int u = 0; u < nb; ++u) {
    const int t = ord[u];
    const DevMaterial& M = c->material(L[t].block);
    ApplyBlock& B = A.b[u];
    B.x = L[t].x;
    B.y = L[t].y;
    B.Ct = M.Ct;
    B.idx = M.idx;
    B.st = L[t].st;
    B.part = L[t].part;
    B.a = L[t].block >= 0 ? L[t].block >> 1 : 0;
    B.c = L[t].block >= 0 ? L[t].block & 1 : 0;
    for (int l = 0; l < 3; ++l) B.ph[l] = L[t].ph[l];
    if (B.part && np_max > part_cap) {
      c->set_error("grid too large for the PCG partial buffers");
      return ST_EINVAL;
    }
  }
  auto launch = [&](int ti, int tj, int chunk) -> int {
    A.tiles_i = (g.L1 + ti - 1) / ti;
    A.tiles_j = (g.L2 + tj - 1) / tj;
    A.chunk = chunk;
    A.per = (int)((long)A.tiles_i * A.tiles_j * ((g.L3 + chunk - 1) / chunk));
    const unsigned grid = (unsigned)((long)A.per * nb);
    if (pal && ti == 16 && tj == 11)
      hipLaunchKernelGGL((apply_stream_kernel<16, 11, true>), dim3(grid),
                         dim3(tile_threads(16, 11)), pal_lds_bytes(c->npal), c->stream, A);
    else if (pal)
      hipLaunchKernelGGL((apply_stream_kernel<TILE_I, TILE_J, true>), dim3(grid),
                         dim3(tile_threads(TILE_I, TILE_J)), pal_lds_bytes(c->npal), c->stream,
                         A);
    else
      hipLaunchKernelGGL((apply_stream_kernel<TILE_I, TILE_J, false>), dim3(grid),
                         dim3(tile_threads(TILE_I, TILE_J)), 0, c->stream, A);
    PBR_HIP(c, hipGetLastError());
    return ST_OK;
  };
  int ti = 0, tj = 0, chunk = 0;
  PBR_TRY(tuned_split(c, g, nb, pal, launch, &ti, &tj, &chunk));
  if (nparts)
    *nparts = (int)((long)((g.L1 + ti - 1) / ti) * ((g.L2 + tj - 1) / tj) *
                    ((g.L3 + PART_G - 1) / PART_G));
  return launch(ti, tj, chunk);
}

int launch_apply(pbr_ctx* c, const Geo& g, int block, double s, const cplx* x, cplx* y,
                 PcgScalars* st, double* part, long part_cap, int* nparts) {
  ApplyLayout L;
  L.block = block;
  for (int l = 0; l < 3; ++l) L.ph[l] = g.ph[l];
  L.x = x;
  L.y = y;
  L.st = st;
  L.part = part;
  return launch_apply_batch(c, g, 1, &L, s, part_cap, nparts);
}
