// The batched persistent hop: descriptors of a batch (lattices and their
// right-hand sides) and the kernel, instantiated per precision in
// bhop_f64.hip, bhop_f32.hip and bhop_f16.hip.
//
// A tile is (lattice, block of 64 sites, set of nw groups of nb right-hand
// sides); a workgroup of nw wavefronts takes one tile at a time, wave w the
// group w of the set, each lane its site for the nb right-hand sides of that
// group, so a link and clover block loaded by a lane serves nb right-hand
// sides from registers and the nw waves of the tile read them at about the
// same time (once from HBM). The tiles of a set of groups of one block are
// consecutive in the tile list, which is dealt to the 8 XCDs in contiguous
// chunks (workgroups reach the XCDs round-robin). Inside a chunk the tiles
// follow a walk chosen by the tuner: linear in the site index, or "slab"
// (each XCD owns the same range of blocks in every time slice and walks the
// slices in order, so that the neighbours in t and z of the sites in flight
// were read shortly before and are still in its L2), optionally with the
// range cut into 2 or 4 sub-ranges walked one after the other. With 12
// right-hand sides a tile's spinors are 12 times a single field's, so the
// walk decides whether neighbour spinors come from L2 or again from HBM.
#pragma once

#include "blas.h"
#include "hopcore.h"
#include "internal.h"

namespace lq {

enum Fld { F_R = 0, F_RHAT, F_P, F_V, F_S, F_T, F_Y, F_X, F_COUNT };

struct BLat {
  Geom g;
  const char* gauge;  // links of the inner precision
  size_t link_stride;
  const void* clov_e;     // A_ee (slot 0) or null
  const void* clov_oinv;  // A_oo^-1 (slot 3) or null
  double kappa;
  int tile0;   // first hop tile of this lattice
  int nsb;     // hop tiles = blocks of 64 sites
  int btile0;  // first blas tile
  int nbb;     // blas blocks (BS sites)
  int nrhs;
  int seg0;
};

struct BSeg {
  void* f[F_COUNT];
  Scal* sc;
  double* partials;
  int lat;
};

struct BHopArgs {
  const BLat* lat;
  const BSeg* seg;
  const int2* tiles;  // (lattice | group set << 8, 64-site block), XCD chunks in order
  int nlat;
  int in_sel, out_sel, own_sel, w_sel;
  int out_parity;
  int clov_slot;      // 0: A_ee, 3: A_oo^-1
  int scale_mode;     // 0: 1, 1: -kappa^2
  int bound[9];       // XCD chunk boundaries of the hop tile list
};

// Launch shape of the batched hop: nb right-hand sides per lane, nw wavefronts
// (groups) per workgroup, nslot workgroups per XCD (the grid is 8 nslot
// workgroups), the tile walk (0 linear, 1 slab, 2 and 3 slab in 2 or 4
// sub-ranges) and nt = 1 for non-temporal
// (streaming) loads of the links and clover blocks.
struct BShape {
  int nb = 4, nw = 3, nslot = 256, walk = 1, nt = 0;
};

constexpr int BHOP_MAX_WAVES = 8;

__device__ inline int find_lat(const BLat* lat, int nlat, int tile, bool blas) {
  int l = 0;
  for (int k = 1; k < nlat; ++k)
    if (tile >= (blas ? lat[k].btile0 : lat[k].tile0)) l = k;
  return l;
}

template <int P, int EPI, bool CLOV, int RED, bool NT, int NB>
__global__ void __launch_bounds__(64 * BHOP_MAX_WAVES) k_bhop(BHopArgs b) {
  constexpr int NR = RED == RED_DOT ? 2 : (RED == RED_TS ? 3 : 0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, nslot = gridDim.x >> 3;
  for (int t = b.bound[xcd] + slot; t < b.bound[xcd + 1]; t += nslot) {
    const int2 tl = b.tiles[t];
    const BLat& L = b.lat[tl.x & 0xff];
    const int sb = tl.y;
    const int grp = (tl.x >> 8) * nw + wv;
    if (grp * NB >= L.nrhs) continue;
    const size_t i = (size_t)sb * SB + lane;
    MultiPtrs<NB> m;
    m.act = 0u;
    int segs[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int r = grp * NB + q;
      segs[q] = -1;
      m.in[q] = nullptr;
      m.out[q] = nullptr;
      m.own[q] = nullptr;
      m.w[q] = nullptr;
      if (r < L.nrhs) {
        const BSeg& S = b.seg[L.seg0 + r];
        segs[q] = L.seg0 + r;
        if (!S.sc->done) m.act |= 1u << q;  // uniform over the wavefront
        m.in[q] = S.f[b.in_sel];
        m.out[q] = S.f[b.out_sel];
        m.own[q] = b.own_sel >= 0 ? S.f[b.own_sel] : nullptr;
        m.w[q] = b.w_sel >= 0 ? S.f[b.w_sel] : nullptr;
      }
    }
    if (m.act == 0u) continue;
    HopArgs a;
    a.in = nullptr;
    a.out = nullptr;
    a.gauge = L.gauge;
    a.link_stride = L.link_stride;
    a.clov = b.clov_slot == 0 ? L.clov_e : L.clov_oinv;
    a.xown = nullptr;
    a.w = nullptr;
    a.partials = nullptr;
    a.skip = nullptr;
    a.scale = b.scale_mode == 0 ? 1.0 : -L.kappa * L.kappa;
    a.g = L.g;
    a.p = b.out_parity;
    a.remap = 0;
    a.hz = 0;
    double red[NB][3];
#pragma unroll
    for (int q = 0; q < NB; ++q) red[q][0] = red[q][1] = red[q][2] = 0.0;
    if (i < (size_t)L.g.vh) hop_site_multi<P, EPI, CLOV, RED, NT, NB>(a, m, i, red);
    if constexpr (NR > 0) {
      // per right-hand side: the wavefront's sum (fixed butterfly order) is
      // the partial of this 64-site block
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (!((m.act >> q) & 1u)) continue;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          double v = red[q][k];
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
          if (lane == 0) b.seg[segs[q]].partials[(size_t)sb * NR + k] = v;
        }
      }
    }
  }
}

// Enqueue one batched hop of storage precision P (instantiated in
// bhop_f{64,32,16}.hip): epi / red / clov select the epilogue as in the
// single-field hop, sh.nb the right-hand sides per lane (1..4; 1..2 in FP64).
template <int P>
int launch_bhop(const BHopArgs& a, const BShape& sh, int epi, int red, bool clov, hipStream_t s);

}  // namespace lq

// One precision's instantiations (expanded in the bhop_f*.hip files).
#define LQ_BHOP_LAUNCH_EPI(P, NT, NB)                                                                         \
  {                                                                                                           \
    const dim3 grid(8 * sh.nslot), block(64 * sh.nw);                                                         \
    if (epi == EPI_SCALE_CLOV) {                                                                              \
      if (clov) hipLaunchKernelGGL((k_bhop<P, EPI_SCALE_CLOV, true, RED_NONE, NT, NB>), grid, block, 0, s, a); \
      else hipLaunchKernelGGL((k_bhop<P, EPI_SCALE, false, RED_NONE, NT, NB>), grid, block, 0, s, a);          \
    } else if (red == RED_DOT) {                                                                              \
      if (clov) hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, true, RED_DOT, NT, NB>), grid, block, 0, s, a);        \
      else hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, false, RED_DOT, NT, NB>), grid, block, 0, s, a);            \
    } else {                                                                                                  \
      if (clov) hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, true, RED_TS, NT, NB>), grid, block, 0, s, a);         \
      else hipLaunchKernelGGL((k_bhop<P, EPI_XPAY, false, RED_TS, NT, NB>), grid, block, 0, s, a);             \
    }                                                                                                         \
    return hipGetLastError() == hipSuccess ? LQCD_OK : set_error(LQCD_EHIP, "batched hop launch failed");    \
  }
#define LQ_BHOP_LAUNCH_NB(P, NB)             \
  if (sh.nb == NB) {                         \
    if (sh.nt) LQ_BHOP_LAUNCH_EPI(P, true, NB) \
    else LQ_BHOP_LAUNCH_EPI(P, false, NB)      \
  }
